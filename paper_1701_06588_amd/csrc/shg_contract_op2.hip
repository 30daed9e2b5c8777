#define SHG_OP 2
#include "shg_contract.inc"
