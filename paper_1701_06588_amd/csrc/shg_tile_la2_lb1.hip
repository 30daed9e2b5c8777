// k_tile instantiations for class (la, lb) = (2, 1), without and with derivatives
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la2_lb1()
{
    static const tile_fn t[2] = {&launch_tile<2, 1, false>, &launch_tile<2, 1, true>};
    return t;
}
}  // namespace shg
