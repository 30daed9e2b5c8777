// k_tile instantiations for class (la, lb) = (9, 3), without and with derivatives
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la9_lb3()
{
    static const tile_fn t[2] = {&launch_tile<9, 3, false>, &launch_tile<9, 3, true>};
    return t;
}
}  // namespace shg
