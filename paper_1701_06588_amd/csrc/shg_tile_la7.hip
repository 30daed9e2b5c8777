#define SHG_LA 7
#define SHG_LBMAX 3
#include "shg_tile.inc"
