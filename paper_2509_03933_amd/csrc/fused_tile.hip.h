// The fused on-chip tile (load -> Stage A -> Stage B -> Stage C -> store) as a
// device function, used by the generic one-tile-per-block kernel (fused.hip).
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

// Stage B replaced by the PDD approximation (Sun's parallel diagonally
// dominant method, which the paper uses for its momentum solves, Sec. 5.1).
// A partition's two interface rows, solved for its own first and last
// unknowns, give the spike form
//   X_first = xf~ - vf X_left - wf X_right,   X_last = xl~ - vl X_left - wl X_right
// (X_left: the previous partition's last unknown, X_right: the next one's
// first; with D = 1 - fc la: xf~ = (fd - fc ld)/D, vf = fa/D, wf = -fc lc/D,
// xl~ = (ld - la fd)/D, vl = -la fa/D, wl = lc/D).  At each interface the
// couplings to the far side (vl of the left partition, wf of the right one:
// spike tips that decay geometrically with the partition length for a
// diagonally dominant matrix) are dropped, leaving independent 2 x 2 systems
// in (X_last of p, X_first of p+1); each lane solves the two interfaces it
// touches from its neighbours' values (one LDS exchange) and applies the
// spike form.  One partition: exact.  LDS: 4 x S x P doubles.  Every thread
// of the block calls it.
__device__ __forceinline__ void pdd_interface(double *lds, int S, int s, int p, int P, Iface f,
                                              double &x_first, double &x_last, bool &bad) {
    const double D = 1.0 - f.fc * f.la;
    bad |= dev::bad_pivot(D);
    const double iD = dev::recip(D);
    const double xtf = (f.fd - f.fc * f.ld) * iD, vf = f.fa * iD, wf = -f.fc * f.lc * iD;
    const double xtl = (f.ld - f.la * f.fd) * iD, vl = -f.la * f.fa * iD, wl = f.lc * iD;
    const int SP = S * P;
    double *XTF = lds, *VF = lds + SP, *XTL = lds + 2 * SP, *WL = lds + 3 * SP;
    const int q = p * S + s;
    __syncthreads();   // the LDS is free
    XTF[q] = xtf;
    VF[q] = vf;
    XTL[q] = xtl;
    WL[q] = wl;
    __syncthreads();
    double left = 0.0, right = 0.0;
    if (p > 0) {         // interface p-1 | p: the previous partition's last unknown
        const double xtl_m = XTL[q - S], wl_m = WL[q - S];
        const double det = 1.0 - wl_m * vf;
        bad |= dev::bad_pivot(det);
        left = (xtl_m - wl_m * xtf) * dev::recip(det);
    }
    if (p < P - 1) {     // interface p | p+1: the next partition's first unknown
        const double xtf_p = XTF[q + S], vf_p = VF[q + S];
        const double det = 1.0 - wl * vf_p;
        bad |= dev::bad_pivot(det);
        right = (xtf_p - vf_p * xtl) * dev::recip(det);
    }
    x_first = xtf - vf * left - wf * right;
    x_last = xtl - vl * left - wl * right;
}

}  // namespace fused_detail
using namespace fused_detail;

// One tile of the fused solve: systems k0 .. k0+S-1 of `map`, S*P lanes of the
// calling block, M rows per lane.  PDD: Stage B by the PDD approximation
// (pdd_interface) instead of the exact interface solve.  Every thread
// of the block must call it.
template <typename T, int M, bool LIKE_D, bool SHIFT, bool CONTIG, bool PDD>
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
        const int pitch = P * (M + 1) + 1;
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
        if constexpr (LIKE_D) {
            // the four arrays' loads in flight together, then through the
            // staging buffer one after the other
            dev::stage_in4_sw<T, M>(stg, tsys, A, B, C, d, S, R, pitch, invR, s, p, av, bv, cv, dv);
        } else {
            dev::stage_in_sw<T, M>(stg, tsys, d, Ident<T>::d, S, R, pitch, invR, s, p, dv);
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
    if constexpr (PDD)
        pdd_interface(lds, S, s, p, P, f, xf, xl, bad);
    else if (P <= 64 && (P & (P - 1)) == 0)
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
        const int pitch = P * (M + 1) + 1;
        T *stg = reinterpret_cast<T *>(lds);
        const size_t stg_bytes = ((size_t)S * pitch * sizeof(T) + 15) & ~(size_t)15;
        const size_t pcr_bytes = dev::pcr_lds_bytes(S, P);
        TileSysLds *tsys = reinterpret_cast<TileSysLds *>(
            reinterpret_cast<char *>(lds) + (stg_bytes > pcr_bytes ? stg_bytes : pcr_bytes));
        dev::stage_out_sw<T, M>(stg, tsys, x, S, R, pitch, 1.0f / (float)R, s, p, dv);
    }
    if (bad && sys.valid) atomicOr(err, 1);
}


// LDS layout of the fused tile: [0, region0) staging (contiguous rows) or the
// Stage B scratch, whichever is larger; the contiguous-row system table; and,
// for a shared operator held in LDS, its 3 x P*M coefficient rows.  The
// generic tile stages with each lane's rows M+1 slots apart (sw, pitch
// P*(M+1)+1), the shared-operator tile with pitch P*M+1.
__host__ __device__ inline size_t fused_region0(size_t esz, int S, int P, int M, bool contig,
                                                bool sw = false) {
    const size_t pcr = dev::pcr_lds_bytes(S, P);
    if (!contig) return pcr;
    const size_t pitch = sw ? (size_t)P * (M + 1) + 1 : (size_t)P * M + 1;
    const size_t stg = ((size_t)S * pitch * esz + 15) & ~(size_t)15;
    return stg > pcr ? stg : pcr;
}

__host__ __device__ inline size_t fused_co_offset(size_t esz, int S, int P, int M, bool contig) {
    const size_t tsys = contig ? (size_t)S * 16 : 0;
    return (fused_region0(esz, S, P, M, contig) + tsys + 15) & ~(size_t)15;
}

// Fused tile of a shared operator (optionally with a per-system diagonal
// shift): the tile's coefficient rows go to LDS once per block, loaded ahead
// of the right-hand sides, and each lane keeps only d^, a^ and c^ of its M
// rows in registers (three values per row instead of four), which doubles
// the blocks a CU holds.  Same arithmetic as fused_tile.  Every thread of
// the block must call it.
template <typename T, int M, bool SHIFT, bool CONTIG, bool PDD>
__device__ __forceinline__ void fused_tile_co(const SysMap &map, const Coef &coef, const T *d, T *x,
                                              int S_log2, int P, int64_t k0, int *err, double *lds) {
    const int tid = threadIdx.x;
    const int S = 1 << S_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int R = P * M;
    const LaneSys sys = dev::lane_system(map, k0 + s);
    const int rows_here = (int)(sys.nrows - r0 < 0 ? 0 : (sys.nrows - r0 > M ? M : sys.nrows - r0));
    char *base = reinterpret_cast<char *>(lds);
    T *CO = reinterpret_cast<T *>(base + fused_co_offset(sizeof(T), S, P, M, CONTIG));

    // coefficient rows first, then the right-hand sides (in flight while the
    // rows go to LDS)
    constexpr int CR = 2;
    dev::RowRegs<CR> rr;
    dev::rows_prefetch<T, CR>(coef, map.n, rr);
    __builtin_amdgcn_sched_barrier(0);
    T dv[M];
    T *stg = reinterpret_cast<T *>(lds);
    TileSysLds *tsys = reinterpret_cast<TileSysLds *>(base + fused_region0(sizeof(T), S, P, M, CONTIG));
    const float invR = 1.0f / (float)R;
    if constexpr (!CONTIG) {
        // branch-free, so the loads form one run behind the coefficient rows:
        // the row index stops at the system's last row (a lane past the last
        // system reads the array's start); padding rows are zeroed below
        const int64_t rs = map.row_stride;
        const int64_t last = sys.nrows > 0 ? sys.nrows - 1 : 0;
        const int64_t first = r0 < last ? r0 : last;
        const int adv = (int)(last - first < M ? last - first : M);
        int64_t idx = (sys.valid ? sys.base : 0) + first * rs;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            dv[j] = d[idx];
            idx += j < adv ? rs : 0;
        }
    } else {
        if (tid < S) {
            const LaneSys q = dev::lane_system(map, k0 + tid);
            tsys[tid].base = q.base;
            tsys[tid].nrows = q.nrows;
        }
        __syncthreads();
        dev::stage_load<T, M>(tsys, d, S, R, invR, dv);
    }
    T sh = T(0);
    if constexpr (SHIFT) {
        sh = ((const T *)coef.shift)[sys.valid ? sys.id : 0];
        if (!sys.valid) sh = T(0);
    }
    dev::rows_commit<T, CR, T>(CO, coef, map.n, R, rr);
    if constexpr (!CONTIG) {
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j >= rows_here) dv[j] = T(0);
    }
    if constexpr (CONTIG) {
        T ld[M];
#pragma unroll
        for (int j = 0; j < M; ++j) ld[j] = dv[j];
        dev::stage_put<T, M>(stg, tsys, Ident<T>::d, S, R, R + 1, invR, s, r0, ld, dv);
    }

    bool bad = false;
    T ah[M], ch[M];
    const Iface f = dev::reduce_partition_rows<T, M, SHIFT>(CO + r0, CO + R + r0, CO + 2 * R + r0, sh,
                                                            rows_here, ah, ch, dv, bad);
    double xf, xl;
    if constexpr (PDD)
        pdd_interface(lds, S, s, p, P, f, xf, xl, bad);
    else if (P <= 64 && (P & (P - 1)) == 0)
        dev::pcr_interface_wave(lds, S, s, p, P, __builtin_ctz(P), f, xf, xl, bad);
    else
        dev::pcr_interface(lds, S, s, p, P, f, xf, xl, bad);
    dev::substitute_partition<T, M>(ah, ch, dv, xf, xl);

    if constexpr (!CONTIG) {
        const int64_t off0 = sys.base + (int64_t)r0 * map.row_stride;
        const int64_t rs = map.row_stride;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < rows_here) x[off0 + j * rs] = dv[j];
    } else {
        dev::stage_out<T, M>(stg, tsys, x, S, R, R + 1, invR, s, r0, dv);
    }
    if (bad && sys.valid) atomicOr(err, 1);
}

}  // namespace tdma
