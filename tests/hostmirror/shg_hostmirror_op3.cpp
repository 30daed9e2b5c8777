#define SHG_OP 3
#include "shg_hostmirror_op.inc"
