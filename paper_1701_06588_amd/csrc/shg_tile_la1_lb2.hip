// k_tile instantiations for class (la, lb) = (1, 2), without and with derivatives
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la1_lb2()
{
    static const tile_fn t[2] = {&launch_tile<1, 2, false>, &launch_tile<1, 2, true>};
    return t;
}
}  // namespace shg
