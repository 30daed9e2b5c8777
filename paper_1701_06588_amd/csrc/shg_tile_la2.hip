#define SHG_LA 2
#define SHG_LBMAX 4
#include "shg_tile.inc"
