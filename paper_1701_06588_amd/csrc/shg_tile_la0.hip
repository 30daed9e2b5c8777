#define SHG_LA 0
#include "shg_tile.inc"
