// persistent kernel instantiation, derivatives = false
#include "shg_persist.h"
namespace shg {
void persist_entry_d0(int group, persist_fn *f, persist_occ_fn *occ)
{
    switch (group) {
    case PG_LIGHT:
        *f = &launch_persist<false, PG_LIGHT>;
        *occ = &persist_occupancy<false, PG_LIGHT>;
        break;
    case PG_HEAVY:
        *f = &launch_persist<false, PG_HEAVY>;
        *occ = &persist_occupancy<false, PG_HEAVY>;
        break;
    default:
        *f = &launch_persist<false, PG_ALL>;
        *occ = &persist_occupancy<false, PG_ALL>;
    }
}
}  // namespace shg
