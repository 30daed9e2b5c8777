#define SHG_OP 4
#include "shg_hostmirror_op.inc"
