#define SHG_LA 3
#define SHG_LBMAX 4
#include "shg_tile.inc"
