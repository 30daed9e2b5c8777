#define SHG_OP 1
#include "shg_contract.inc"
