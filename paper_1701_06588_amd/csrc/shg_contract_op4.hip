#define SHG_OP 4
#include "shg_contract.inc"
