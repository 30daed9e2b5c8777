#define SHG_OP 2
#include "shg_hostmirror_op.inc"
