#define SHG_OP 0
#include "shg_hostmirror_op.inc"
