#define SHG_LA 3
#include "shg_assemble.inc"
