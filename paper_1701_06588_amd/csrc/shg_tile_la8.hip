#define SHG_LA 8
#define SHG_LBMAX 3
#include "shg_tile.inc"
