// shg_persist.h -- persistent, class-binned kernel of the batched path.
//
// One launch evaluates every tile of a plan (tiles of 64 pairs, the compiled
// tile schedule of each class): each workgroup repeatedly takes
// the next tile index from a device counter (one atomic per tile), reads the
// tile's class and range from the work queue and runs the class's tile code
// (tile_pairs, shared with the per-class kernels). The index of the following
// tile is requested when a tile starts and handed over through LDS once phase
// 1 has waited for its loads, so the atomic's round trip is hidden. All
// classes of one derivative flavour live in this one kernel; the queue (built
// by the plan) alternates heavy and light tiles. Every workgroup exits once the
// counter passes the number of tiles.
#pragma once
#include "shg_kernels.h"

namespace shg {

struct QTile {
    int32_t cls;      // la * 5 + lb
    int32_t count;    // pairs in the tile (<= shape.tp)
    int64_t start;    // first sorted position
};

// dynamic LDS limit of the persistent kernel (160 KiB minus its static LDS)
constexpr int PERSIST_MAX_SMEM = 160 * 1024 - 256;

// Class groups: one kernel may hold every class (PG_ALL) or only the light
// (la + lb <= 4) or the heavy ones. A kernel's register count is that of the
// union of its classes' bodies, so the light classes, run by a kernel of their
// own, keep three workgroups per CU where the all-class kernel keeps two.
enum { PG_ALL = 0, PG_LIGHT = 1, PG_HEAVY = 2 };
constexpr int PG_LIGHT_MAX = 4;   // light: la + lb <= 4
constexpr bool persist_has(int group, int la, int lb)
{
    return group == PG_ALL || (group == PG_LIGHT) == (la + lb <= PG_LIGHT_MAX);
}

// ntiles < 0: the number of tiles is read from counter[1] (written by an
// earlier kernel of the same stream, e.g. a screening stage)
template <bool D, int GROUP>
__global__ __launch_bounds__(TILE_THREADS) void k_persist(TileArgs a, const QTile *__restrict__ q, int ntiles,
                                                          int *counter)
{
    extern __shared__ __align__(16) char smem[];
    // tile index of iteration k in s_t[k & 1]: written by thread 0 during
    // iteration k - 1 (after phase 1), read by all after that tile's last barrier
    __shared__ int s_t[2];
    if (threadIdx.x == 0) s_t[0] = atomicAdd(counter, 1);
    const int nt = ntiles >= 0 ? ntiles : counter[1];
    __syncthreads();
    for (int k = 0;; ++k) {
        const int t = s_t[k & 1];
        if (t >= nt) break;
        int nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(counter, 1);
        const auto hand_over = [&]() {
            if (threadIdx.x == 0) s_t[(k + 1) & 1] = nxt;
        };
        const QTile tile = q[t];
        static_for<0, NCLASS>([&](auto CC) {
            constexpr int C = decltype(CC)::value;
            constexpr int LA = C / (LMAX + 1), LB = C % (LMAX + 1);
            if constexpr (persist_has(GROUP, LA, LB))
                if (tile.cls == C)
                    tile_pairs<LA, LB, D, sched_rows(LA, LB, D)>(a, tile.start, tile.count, TileShape{64, 1}, smem,
                                                                 hand_over);
        });
    }
}

typedef void (*persist_fn)(hipStream_t, int grid, size_t smem, const TileArgs &, const QTile *, int, int *);
typedef int (*persist_occ_fn)(size_t smem);

template <bool D, int GROUP>
void launch_persist(hipStream_t s, int grid, size_t smem, const TileArgs &a, const QTile *q, int ntiles, int *counter)
{
    hipLaunchKernelGGL((k_persist<D, GROUP>), dim3(grid), dim3(TILE_THREADS), smem, s, a, q, ntiles, counter);
}

// also raises the kernel's dynamic-LDS limit (done here, before any graph
// capture, rather than inside the launch)
template <bool D, int GROUP>
int persist_occupancy(size_t smem)
{
    if (hipFuncSetAttribute((const void *)k_persist<D, GROUP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            PERSIST_MAX_SMEM) != hipSuccess)
        (void)hipGetLastError();   // the launch then fails and reports it; leave nothing sticky here
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<D, GROUP>, TILE_THREADS, smem);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // do not leave a sticky error behind
        return 1;
    }
    return nb > 0 ? nb : 1;
}

// defined in shg_persist_d0.hip / shg_persist_d1.hip: the launch and occupancy
// functions of class group `group` (PG_ALL, PG_LIGHT, PG_HEAVY)
void persist_entry_d0(int group, persist_fn *f, persist_occ_fn *occ);
void persist_entry_d1(int group, persist_fn *f, persist_occ_fn *occ);

}  // namespace shg
