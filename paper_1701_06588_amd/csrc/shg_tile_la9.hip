#define SHG_LA 9
#define SHG_LBMAX 3
#include "shg_tile.inc"
