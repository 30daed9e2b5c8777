#define SHG_LA 1
#define SHG_LBMAX 4
#include "shg_tile.inc"
