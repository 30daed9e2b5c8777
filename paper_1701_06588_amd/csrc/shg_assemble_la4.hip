#define SHG_LA 4
#include "shg_assemble.inc"
