// Fused on-chip solve: load -> Stage A -> Stage B (PCR) -> Stage C -> store,
// one launch, intermediates only in registers and LDS.
#include "tile.hip.h"

namespace tdma {
namespace {

using dev::Iface;
using dev::LaneSys;
using dev::Ident;
using dev::TileSysLds;
using dev::stage_in;
using dev::stage_out;

// Largest block for M rows per lane: lanes holding >= 128 bytes per array
// get up to 256 VGPRs (2+ waves/SIMD) instead of the 128 a 1024-block allows.
template <typename T, int M>
constexpr int fused_max_threads() { return (int)sizeof(T) * M >= 128 ? 512 : 1024; }

template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG>
__global__ void __launch_bounds__((fused_max_threads<T, M>()))
k_fused(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P, int *err) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int S = 1 << S_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t k0 = (int64_t)blockIdx.x << S_log2;
    if (map.count && k0 >= dev::launch_nsys(map)) return;   // whole tile past a device count
    const LaneSys sys = dev::lane_system(map, k0 + s);
    const T *__restrict__ A = (const T *)coef.a;
    const T *__restrict__ B = (const T *)coef.b;
    const T *__restrict__ C = (const T *)coef.c;

    T av[M], bv[M], cv[M], dv[M];
    const int rows_here = (int)(sys.nrows - r0 < 0 ? 0 : (sys.nrows - r0 > M ? M : sys.nrows - r0));
    if constexpr (!CONTIG) {
        const int64_t off0 = sys.base + (int64_t)r0 * map.row_stride;
        const int64_t rs = map.row_stride;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < rows_here) {
                const int64_t idx = off0 + j * rs;
                dv[j] = d[idx];
                if constexpr (LIKE_D) {
                    av[j] = A[idx]; bv[j] = B[idx]; cv[j] = C[idx];
                } else {
                    av[j] = A[r0 + j]; bv[j] = B[r0 + j]; cv[j] = C[r0 + j];
                }
            } else {
                av[j] = Ident<T>::a; bv[j] = Ident<T>::b; cv[j] = Ident<T>::c; dv[j] = Ident<T>::d;
            }
        }
    } else {
        const int R = P * M;
        const int pitch = R + 1;
        T *stg = reinterpret_cast<T *>(lds);
        const size_t stg_bytes = ((size_t)S * pitch * sizeof(T) + 15) & ~(size_t)15;
        const size_t pcr_bytes = dev::pcr_lds_bytes(S, P);
        TileSysLds *tsys = reinterpret_cast<TileSysLds *>(
            reinterpret_cast<char *>(lds) + (stg_bytes > pcr_bytes ? stg_bytes : pcr_bytes));
        if (tid < S) {
            const LaneSys q = dev::lane_system(map, k0 + tid);
            tsys[tid].base = q.base;
            tsys[tid].nrows = q.nrows;
        }
        const float invR = 1.0f / (float)R;
        stage_in<T, M>(stg, tsys, d, Ident<T>::d, S, R, pitch, invR, s, r0, dv);
        if constexpr (LIKE_D) {
            stage_in<T, M>(stg, tsys, A, Ident<T>::a, S, R, pitch, invR, s, r0, av);
            stage_in<T, M>(stg, tsys, B, Ident<T>::b, S, R, pitch, invR, s, r0, bv);
            stage_in<T, M>(stg, tsys, C, Ident<T>::c, S, R, pitch, invR, s, r0, cv);
        } else {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int64_t r = r0 + j;
                if (r < sys.nrows) {
                    av[j] = A[r]; bv[j] = B[r]; cv[j] = C[r];
                } else {
                    av[j] = Ident<T>::a; bv[j] = Ident<T>::b; cv[j] = Ident<T>::c;
                }
            }
        }
    }
    if constexpr (SHIFT) {
        if (sys.valid) {
            const T sh = ((const T *)coef.shift)[sys.id];
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (r0 + j < sys.nrows) bv[j] += sh;
        }
    }
    // the matrix has no a_0 and no c_{n-1}
    if (r0 == 0) av[0] = T(0);
#pragma unroll
    for (int j = 0; j < M; ++j)
        if (r0 + j == sys.nrows - 1) cv[j] = T(0);

    bool bad = false;
    const Iface f = dev::reduce_partition<T, M>(av, bv, cv, dv, bad);
    double xf, xl;
    if (P <= 64 && (P & (P - 1)) == 0)
        dev::pcr_interface_wave(lds, S, s, p, P, __builtin_ctz(P), f, xf, xl, bad);
    else
        dev::pcr_interface(lds, S, s, p, P, f, xf, xl, bad);
    dev::substitute_partition<T, M>(av, cv, dv, xf, xl);

    if constexpr (!CONTIG) {
        const int64_t off0 = sys.base + (int64_t)r0 * map.row_stride;
        const int64_t rs = map.row_stride;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < rows_here) x[off0 + j * rs] = dv[j];
    } else {
        const int R = P * M;
        const int pitch = R + 1;
        T *stg = reinterpret_cast<T *>(lds);
        const size_t stg_bytes = ((size_t)S * pitch * sizeof(T) + 15) & ~(size_t)15;
        const size_t pcr_bytes = dev::pcr_lds_bytes(S, P);
        TileSysLds *tsys = reinterpret_cast<TileSysLds *>(
            reinterpret_cast<char *>(lds) + (stg_bytes > pcr_bytes ? stg_bytes : pcr_bytes));
        stage_out<T, M>(stg, tsys, x, S, R, pitch, 1.0f / (float)R, s, r0, dv);
    }
    if (bad && sys.valid) atomicOr(err, 1);
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
