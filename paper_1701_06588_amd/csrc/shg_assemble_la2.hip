#define SHG_LA 2
#include "shg_assemble.inc"
