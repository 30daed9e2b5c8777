#define SHG_LA 3
#include "shg_tile.inc"
