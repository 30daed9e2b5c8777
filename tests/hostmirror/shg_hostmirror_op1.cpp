#define SHG_OP 1
#include "shg_hostmirror_op.inc"
