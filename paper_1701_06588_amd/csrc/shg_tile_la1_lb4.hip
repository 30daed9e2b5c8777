// k_tile instantiations for class (la, lb) = (1, 4), without and with derivatives
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la1_lb4()
{
    static const tile_fn t[2] = {&launch_tile<1, 4, false>, &launch_tile<1, 4, true>};
    return t;
}
}  // namespace shg
