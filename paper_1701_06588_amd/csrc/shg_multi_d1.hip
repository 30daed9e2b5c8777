// multi-operator persistent kernel instantiation, derivatives = true
#include "shg_multi.h"
namespace shg {
void multi_entry_d1(multi_fn *f, multi_occ_fn *occ)
{
    *f = &launch_multi<true>;
    *occ = &multi_occupancy<true>;
}
}  // namespace shg
