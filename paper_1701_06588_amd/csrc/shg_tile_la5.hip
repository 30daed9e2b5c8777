#define SHG_LA 5
#define SHG_LBMAX 3
#include "shg_tile.inc"
