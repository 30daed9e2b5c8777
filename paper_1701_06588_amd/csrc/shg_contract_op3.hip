#define SHG_OP 3
#include "shg_contract.inc"
