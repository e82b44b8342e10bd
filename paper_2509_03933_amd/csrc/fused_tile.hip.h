// The fused on-chip tile (load -> Stage A -> Stage B -> Stage C -> store) as a
// device function, shared by the one-tile-per-block kernel (fused.hip) and
// the persistent work-queue kernel (persist.hip).
#pragma once
#include "tile.hip.h"

namespace tdma {
namespace fused_detail {

using dev::Iface;
using dev::LaneSys;
using dev::Ident;
using dev::TileSysLds;
using dev::stage_out;

// Largest block for M rows per lane: lanes holding >= 128 bytes per array
// get up to 256 VGPRs (2+ waves/SIMD) instead of the 128 a 1024-block allows.
template <typename T, int M>
constexpr int fused_max_threads() { return (int)sizeof(T) * M >= 128 ? 512 : 1024; }

}  // namespace fused_detail
using namespace fused_detail;

// One tile of the fused solve: systems k0 .. k0+S-1 of `map`, S*P lanes of the
// calling block, M rows per lane.  Every thread of the block must call it.
template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG>
__device__ __forceinline__ void fused_tile(const SysMap &map, const Coef &coef, const T *d, T *x,
                                           int S_log2, int P, int64_t k0, int *err, double *lds) {

    const int tid = threadIdx.x;
    const int S = 1 << S_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
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
        if constexpr (!LIKE_D) {
            // shared coefficient rows (clamped into the system, padding below)
            const int64_t last = sys.nrows > 0 ? sys.nrows - 1 : 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int64_t r = r0 + j < last ? r0 + j : last;
                av[j] = A[r]; bv[j] = B[r]; cv[j] = C[r];
            }
        }
        // one array at a time through the staging buffer
        dev::stage_in<T, M>(stg, tsys, d, Ident<T>::d, S, R, pitch, invR, s, r0, dv);
        if constexpr (LIKE_D) {
            dev::stage_in<T, M>(stg, tsys, A, Ident<T>::a, S, R, pitch, invR, s, r0, av);
            dev::stage_in<T, M>(stg, tsys, B, Ident<T>::b, S, R, pitch, invR, s, r0, bv);
            dev::stage_in<T, M>(stg, tsys, C, Ident<T>::c, S, R, pitch, invR, s, r0, cv);
        } else {
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (r0 + j >= sys.nrows) {
                    av[j] = Ident<T>::a; bv[j] = Ident<T>::b; cv[j] = Ident<T>::c;
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


}  // namespace tdma
