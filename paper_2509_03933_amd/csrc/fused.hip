// Fused on-chip solve: load -> Stage A -> Stage B (PCR) -> Stage C -> store,
// one launch, intermediates only in registers and LDS.
#include "fused_tile.hip.h"

namespace tdma {

namespace {

// CO: a shared operator whose coefficient rows are held in LDS (fused_tile_co).
// PDD: Stage B by the PDD approximation (its own instantiations, so that the
// exact kernels keep their register allocation).
template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG, bool CO, bool PDD>
__global__ void __launch_bounds__((fused_max_threads<T, M>()))
k_fused(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P, int *err) {
    extern __shared__ double lds[];
    const int64_t k0 = dev::xcd_tile(blockIdx.x, gridDim.x) << S_log2;
    if (map.count && k0 >= dev::launch_nsys(map)) return;   // whole tile past a device count
    if constexpr (CO)
        fused_tile_co<T, M, SHIFT, CONTIG, PDD>(map, coef, d, x, S_log2, P, k0, err, lds);
    else
        fused_tile<T, M, LIKE_D, SHIFT, CONTIG, PDD>(map, coef, d, x, S_log2, P, k0, err, lds);
}

// A whole ragged batch of per-row systems in one launch: block b solves tile
// b of a list that the plan orders longest systems first; every tile's
// S*P lanes fill the block, whatever its partition count.
template <typename T, int M>
__global__ void __launch_bounds__((fused_max_threads<T, M>()))
k_fused_tiles(SysMap map, Coef coef, const T *d, T *x, const RaggedTile *tiles, int *err) {
    extern __shared__ double lds[];
    const RaggedTile tl = tiles[blockIdx.x];
    SysMap m = map;
    m.sys_list = map.sys_list + tl.first;
    m.nsys = tl.count;
    m.n = (int64_t)M << tl.P_log2;
    fused_tile<T, M, true, false, true, false>(m, coef, d, x, tl.S_log2, 1 << tl.P_log2, 0, err, lds);
}

template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG, bool CO>
hipError_t launch_t(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                    void *x, int *err, size_t lds, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    if (sh.pdd)
        hipLaunchKernelGGL((k_fused<T, M, LIKE_D, SHIFT, CONTIG, CO, true>), dim3((unsigned)blocks),
                           dim3(sh.threads()), lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2,
                           sh.P, err);
    else
        hipLaunchKernelGGL((k_fused<T, M, LIKE_D, SHIFT, CONTIG, CO, false>), dim3((unsigned)blocks),
                           dim3(sh.threads()), lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2,
                           sh.P, err);
    return hipGetLastError();
}

// Largest LDS footprint for which a shared operator is held in LDS: two
// blocks must still fit a CU.
constexpr size_t kCoLdsLimit = 64 * 1024;

template <typename T, int M>
hipError_t launch_m(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                    void *x, int *err, hipStream_t st) {
    const bool like_d = coef.mode == TDMA_COEF_LIKE_D;
    const bool shift = coef.shift != nullptr;
    const int dtype = sizeof(T) == 8 ? TDMA_F64 : TDMA_F32;
    const size_t lds_co = fused_lds_bytes(dtype, sh, true);
    const bool co = !like_d && lds_co <= kCoLdsLimit;
    const size_t lds = co ? lds_co : fused_lds_bytes(dtype, sh, false);
#define TDMA_DISPATCH(LD, SH, CT, C)                                                         \
    if (like_d == LD && shift == SH && sh.contig == CT && co == C)                           \
        return launch_t<T, M, LD, SH, CT, C>(map, coef, sh, d, x, err, lds, st);
    TDMA_DISPATCH(true, false, false, false)
    TDMA_DISPATCH(true, true, false, false)
    TDMA_DISPATCH(false, false, false, false)
    TDMA_DISPATCH(false, true, false, false)
    TDMA_DISPATCH(true, false, true, false)
    TDMA_DISPATCH(true, true, true, false)
    TDMA_DISPATCH(false, false, true, false)
    TDMA_DISPATCH(false, true, true, false)
    TDMA_DISPATCH(false, false, false, true)
    TDMA_DISPATCH(false, true, false, true)
    TDMA_DISPATCH(false, false, true, true)
    TDMA_DISPATCH(false, true, true, true)
#undef TDMA_DISPATCH
    return hipErrorInvalidValue;
}

}  // namespace

int fused_max_threads(int dtype, int M) {
    const int esz = dtype == TDMA_F64 ? 8 : 4;
    return esz * M >= 128 ? 512 : 1024;
}

bool fused_supported(int dtype, const TileShape &sh) {
    if (sh.P < 1 || sh.S_log2 < 0 || sh.threads() < 1) return false;
    if (sh.threads() > fused_max_threads(dtype, sh.M)) return false;
    if (dtype == TDMA_F64) return sh.M == 4 || sh.M == 8 || sh.M == 16;
    if (dtype == TDMA_F32) return sh.M == 4 || sh.M == 8 || sh.M == 16 || sh.M == 32;
    return false;
}

bool fused_tiles_supported(int dtype, int M) {
    return dtype == TDMA_F64 ? M == 16 : (dtype == TDMA_F32 && (M == 16 || M == 32));
}

hipError_t launch_fused_tiles(int dtype, int M, const SysMap &map, const Coef &coef, const void *d,
                              void *x, const RaggedTile *tiles, int64_t ntiles, int threads,
                              size_t lds, int *err, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (!fused_tiles_supported(dtype, M) || threads > fused_max_threads(dtype, M) ||
        coef.mode != TDMA_COEF_LIKE_D || coef.shift != nullptr || lds > 160 * 1024)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)ntiles), block((unsigned)threads);
    if (dtype == TDMA_F64)
        hipLaunchKernelGGL((k_fused_tiles<double, 16>), grid, block, lds, st, map, coef, (const double *)d,
                           (double *)x, tiles, err);
    else if (M == 16)
        hipLaunchKernelGGL((k_fused_tiles<float, 16>), grid, block, lds, st, map, coef, (const float *)d,
                           (float *)x, tiles, err);
    else
        hipLaunchKernelGGL((k_fused_tiles<float, 32>), grid, block, lds, st, map, coef, (const float *)d,
                           (float *)x, tiles, err);
    return hipGetLastError();
}

size_t fused_lds_bytes(int dtype, const TileShape &sh, bool shared_rows) {
    const int S = 1 << sh.S_log2;
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    if (shared_rows)
        return fused_co_offset(esz, S, sh.P, sh.M, sh.contig) + 3 * (size_t)sh.P * sh.M * esz;
    return fused_region0(esz, S, sh.P, sh.M, sh.contig, true) + (sh.contig ? (size_t)S * 16 : 0);
}

hipError_t launch_fused(int dtype, const SysMap &map, const Coef &coef, const TileShape &sh,
                        const void *d, void *x, int *err, hipStream_t st) {
    if (dtype == TDMA_F64) {
        switch (sh.M) {
            case 4: return launch_m<double, 4>(map, coef, sh, d, x, err, st);
            case 8: return launch_m<double, 8>(map, coef, sh, d, x, err, st);
            case 16: return launch_m<double, 16>(map, coef, sh, d, x, err, st);
        }
    } else if (dtype == TDMA_F32) {
        switch (sh.M) {
            case 4: return launch_m<float, 4>(map, coef, sh, d, x, err, st);
            case 8: return launch_m<float, 8>(map, coef, sh, d, x, err, st);
            case 16: return launch_m<float, 16>(map, coef, sh, d, x, err, st);
            case 32: return launch_m<float, 32>(map, coef, sh, d, x, err, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace tdma
