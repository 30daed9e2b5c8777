// multi-operator persistent kernel instantiation, derivatives = false
#include "shg_multi.h"
namespace shg {
void multi_entry_d0(multi_fn *f, multi_occ_fn *occ)
{
    *f = &launch_multi<false>;
    *occ = &multi_occupancy<false>;
}
}  // namespace shg
