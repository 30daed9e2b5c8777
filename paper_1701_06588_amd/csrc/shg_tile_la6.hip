#define SHG_LA 6
#define SHG_LBMAX 3
#include "shg_tile.inc"
