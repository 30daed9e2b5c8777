#define SHG_LA 4
#include "shg_tile.inc"
