#define SHG_OP 0
#include "shg_contract.inc"
