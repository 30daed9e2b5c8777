// k_tile instantiations for class (la, lb) = (0, 1), without and with derivatives
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la0_lb1()
{
    static const tile_fn t[2] = {&launch_tile<0, 1, false>, &launch_tile<0, 1, true>};
    return t;
}
}  // namespace shg
