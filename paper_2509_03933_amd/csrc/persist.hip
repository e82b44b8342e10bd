// Batching form: one persistent work-queue kernel for a list of solves.
//
// Work items (x/y/z sweeps of a grid, ragged batches split by length class)
// are cut into tiles of the fused solve (fused_tile.hip.h) whose S*P lanes
// fill one 1024-lane block.  A block pops the next tile with an atomic
// counter; tiles are queued in dependency order, so every tile a popped tile
// waits for has already been popped by a running block and the wait always
// ends.  A tile of an item that reads another item's output waits, on the
// device, until that item's completion counter reaches its tile count
// (agent-scope acquire); a finished tile bumps its own item's counter
// (agent-scope release after a block barrier).  Independent tiles (ragged
// systems) are queued between the dependent items to fill the waits.  Every
// wait is bounded: past the limit the block flags an error and continues, so
// no wave can spin forever.  Blocks exit when the queue is empty.
#include "fused_tile.hip.h"
#include "persist.h"

namespace tdma {
namespace {

constexpr int kPersistM = 8;
constexpr unsigned long long kSpinLimit = 1ull << 24;

template <typename T>
__device__ __forceinline__ void run_tile(const WorkDesc &wd, int64_t local, int *err, double *lds) {
    const int64_t k0 = local << wd.S_log2;
    const T *d = (const T *)wd.d;
    T *x = (T *)wd.x;
#define TDMA_P(LD, SH, CT)                                                                      \
    if (wd.like_d == LD && wd.shift == SH && wd.contig == CT) {                                 \
        fused_tile<T, kPersistM, LD, SH, CT>(wd.map, wd.coef, d, x, wd.S_log2, wd.P, k0, err, lds); \
        return;                                                                                 \
    }
    TDMA_P(1, 0, 0)
    TDMA_P(1, 1, 0)
    TDMA_P(0, 0, 0)
    TDMA_P(0, 1, 0)
    TDMA_P(1, 0, 1)
    TDMA_P(1, 1, 1)
    TDMA_P(0, 0, 1)
    TDMA_P(0, 1, 1)
#undef TDMA_P
}

template <typename T>
__global__ void __launch_bounds__(kPersistThreads)
k_persist(const WorkDesc *descs, const WorkSeg *segs, int nsegs, int64_t total_tiles,
          WorkCounters *ctr, int *err) {
    extern __shared__ double lds[];
    __shared__ long long s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (long long)atomicAdd(&ctr->head, 1ull);
        __syncthreads();
        const long long g = s_tile;
        __syncthreads();
        if (g >= total_tiles) break;
        int si = 0;
        while (si + 1 < nsegs && segs[si + 1].global_begin <= g) ++si;
        const WorkSeg sg = segs[si];
        const WorkDesc wd = descs[sg.desc];
        const int64_t local = sg.tile_begin + (g - sg.global_begin);
        if (wd.after >= 0) {
            if (threadIdx.x == 0) {
                const unsigned long long need = (unsigned long long)descs[wd.after].ntiles;
                unsigned long long spins = 0;
                while (__hip_atomic_load(&ctr->done[wd.after], __ATOMIC_ACQUIRE,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit) {
                        atomicOr(err, 2);
                        break;
                    }
                }
            }
            __syncthreads();
        }
        run_tile<T>(wd, local, err, lds);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&ctr->done[sg.desc], 1ull, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_persist_reset(WorkCounters *ctr, int ndesc) {
    const int i = threadIdx.x;
    if (i == 0) ctr->head = 0ull;
    for (int k = i; k < ndesc; k += blockDim.x) ctr->done[k] = 0ull;
}

}  // namespace

int persist_rows_per_lane() { return kPersistM; }

hipError_t persist_occupancy(int dtype, size_t lds, int *blocks_per_cu) {
    if (dtype == TDMA_F64)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persist<double>,
                                                            kPersistThreads, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persist<float>,
                                                        kPersistThreads, lds);
}

hipError_t launch_persist_reset(WorkCounters *ctr, int ndesc, hipStream_t st) {
    hipLaunchKernelGGL(k_persist_reset, dim3(1), dim3(256), 0, st, ctr, ndesc);
    return hipGetLastError();
}

hipError_t launch_persist(int dtype, int grid, size_t lds, const WorkDesc *descs,
                          const WorkSeg *segs, int nsegs, int64_t total_tiles, WorkCounters *ctr,
                          int *err, hipStream_t st) {
    if (dtype == TDMA_F64)
        hipLaunchKernelGGL(k_persist<double>, dim3(grid), dim3(kPersistThreads), lds, st, descs,
                           segs, nsegs, total_tiles, ctr, err);
    else
        hipLaunchKernelGGL(k_persist<float>, dim3(grid), dim3(kPersistThreads), lds, st, descs, segs,
                           nsegs, total_tiles, ctr, err);
    return hipGetLastError();
}

}  // namespace tdma
