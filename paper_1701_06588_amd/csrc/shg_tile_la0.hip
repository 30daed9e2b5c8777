#define SHG_LA 0
#define SHG_LBMAX 4
#include "shg_tile.inc"
