#define SHG_LA 2
#include "shg_tile.inc"
