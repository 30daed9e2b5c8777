// k_tile instantiations for class (la, lb) = (6, 0), without and with derivatives
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la6_lb0()
{
    static const tile_fn t[2] = {&launch_tile<6, 0, false>, &launch_tile<6, 0, true>};
    return t;
}
}  // namespace shg
