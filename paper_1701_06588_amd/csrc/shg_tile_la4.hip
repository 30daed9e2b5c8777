#define SHG_LA 4
#define SHG_LBMAX 4
#include "shg_tile.inc"
