// persistent kernel instantiation, derivatives = true
#include "shg_persist.h"
namespace shg {
void persist_entry_d1(persist_fn *f, persist_occ_fn *occ)
{
    *f = &launch_persist<true>;
    *occ = &persist_occupancy<true>;
}
}  // namespace shg
