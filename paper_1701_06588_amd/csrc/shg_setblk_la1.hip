// k_setblk instantiations for l_a = 1 (every l_b, without and with derivatives)
#include "shg_sets.h"
namespace shg {
const setblk_fn *setblk_table_la1()
{
    static const setblk_fn t[2 * (LMAX + 1)] = {
        &launch_setblk<1, 0, false>, &launch_setblk<1, 0, true>, &launch_setblk<1, 1, false>,
        &launch_setblk<1, 1, true>,  &launch_setblk<1, 2, false>, &launch_setblk<1, 2, true>,
        &launch_setblk<1, 3, false>, &launch_setblk<1, 3, true>,  &launch_setblk<1, 4, false>,
        &launch_setblk<1, 4, true>};
    return t;
}
}  // namespace shg
