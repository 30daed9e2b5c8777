// persistent kernel instantiation, derivatives = false
#include "shg_persist.h"
namespace shg {
void persist_entry_d0(persist_fn *f, persist_occ_fn *occ)
{
    *f = &launch_persist<false>;
    *occ = &persist_occupancy<false>;
}
}  // namespace shg
