// persistent kernel instantiation, derivatives = true
#include "shg_persist.h"
namespace shg {
void persist_entry_d1(int group, persist_fn *f, persist_occ_fn *occ)
{
    switch (group) {
    case PG_LIGHT:
        *f = &launch_persist<true, PG_LIGHT>;
        *occ = &persist_occupancy<true, PG_LIGHT>;
        break;
    case PG_HEAVY:
        *f = &launch_persist<true, PG_HEAVY>;
        *occ = &persist_occupancy<true, PG_HEAVY>;
        break;
    default:
        *f = &launch_persist<true, PG_ALL>;
        *occ = &persist_occupancy<true, PG_ALL>;
    }
}
}  // namespace shg
