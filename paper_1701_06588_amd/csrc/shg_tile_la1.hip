#define SHG_LA 1
#include "shg_tile.inc"
