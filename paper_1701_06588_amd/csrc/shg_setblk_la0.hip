// k_setblk instantiations for l_a = 0 (every l_b, without and with derivatives)
#include "shg_sets.h"
namespace shg {
const setblk_fn *setblk_table_la0()
{
    static const setblk_fn t[2 * (LMAX + 1)] = {
        &launch_setblk<0, 0, false>, &launch_setblk<0, 0, true>, &launch_setblk<0, 1, false>,
        &launch_setblk<0, 1, true>,  &launch_setblk<0, 2, false>, &launch_setblk<0, 2, true>,
        &launch_setblk<0, 3, false>, &launch_setblk<0, 3, true>,  &launch_setblk<0, 4, false>,
        &launch_setblk<0, 4, true>};
    return t;
}
}  // namespace shg
