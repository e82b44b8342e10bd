// Fused on-chip solve: load -> Stage A -> Stage B (PCR) -> Stage C -> store,
// one launch, intermediates only in registers and LDS.
#include "fused_tile.hip.h"

namespace tdma {

namespace {

template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG>
__global__ void __launch_bounds__((fused_max_threads<T, M>()))
k_fused(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P, int *err) {
    extern __shared__ double lds[];
    const int64_t k0 = dev::xcd_tile(blockIdx.x, gridDim.x) << S_log2;
    if (map.count && k0 >= dev::launch_nsys(map)) return;   // whole tile past a device count
    fused_tile<T, M, LIKE_D, SHIFT, CONTIG>(map, coef, d, x, S_log2, P, k0, err, lds);
}

template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG>
hipError_t launch_t(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                    void *x, int *err, size_t lds, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_fused<T, M, LIKE_D, SHIFT, CONTIG>), dim3((unsigned)blocks),
                       dim3(sh.threads()), lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2,
                       sh.P, err);
    return hipGetLastError();
}

template <typename T, int M>
hipError_t launch_m(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                    void *x, int *err, size_t lds, hipStream_t st) {
    const bool like_d = coef.mode == TDMA_COEF_LIKE_D;
    const bool shift = coef.shift != nullptr;
#define TDMA_DISPATCH(LD, SH, CT)                                                            \
    if (like_d == LD && shift == SH && sh.contig == CT)                                      \
        return launch_t<T, M, LD, SH, CT>(map, coef, sh, d, x, err, lds, st);
    TDMA_DISPATCH(true, false, false)
    TDMA_DISPATCH(true, true, false)
    TDMA_DISPATCH(false, false, false)
    TDMA_DISPATCH(false, true, false)
    TDMA_DISPATCH(true, false, true)
    TDMA_DISPATCH(true, true, true)
    TDMA_DISPATCH(false, false, true)
    TDMA_DISPATCH(false, true, true)
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

size_t fused_lds_bytes(int dtype, const TileShape &sh) {
    const size_t S = (size_t)1 << sh.S_log2;
    const size_t pcr = dev::pcr_lds_bytes((int)S, sh.P);
    if (!sh.contig) return pcr;
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    const size_t stg = (S * ((size_t)sh.P * sh.M + 1) * esz + 15) & ~(size_t)15;
    return (stg > pcr ? stg : pcr) + S * 16;
}

hipError_t launch_fused(int dtype, const SysMap &map, const Coef &coef, const TileShape &sh,
                        const void *d, void *x, int *err, hipStream_t st) {
    const size_t lds = fused_lds_bytes(dtype, sh);
    if (dtype == TDMA_F64) {
        switch (sh.M) {
            case 4: return launch_m<double, 4>(map, coef, sh, d, x, err, lds, st);
            case 8: return launch_m<double, 8>(map, coef, sh, d, x, err, lds, st);
            case 16: return launch_m<double, 16>(map, coef, sh, d, x, err, lds, st);
        }
    } else if (dtype == TDMA_F32) {
        switch (sh.M) {
            case 4: return launch_m<float, 4>(map, coef, sh, d, x, err, lds, st);
            case 8: return launch_m<float, 8>(map, coef, sh, d, x, err, lds, st);
            case 16: return launch_m<float, 16>(map, coef, sh, d, x, err, lds, st);
            case 32: return launch_m<float, 32>(map, coef, sh, d, x, err, lds, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace tdma
