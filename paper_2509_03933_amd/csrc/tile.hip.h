// Device building blocks of the on-chip partitioned solve (gfx950).
//
// A tile is S systems x P partitions; lane (p, s) = threadIdx.x = p*S + s holds
// rows p*M .. p*M+M-1 of system s in registers.  Consecutive lanes hold the
// same row of consecutive systems, so for y/z lines (systems adjacent in
// memory) every row load is one contiguous S-element segment.
//
// Math (the paper's Stage A / B / C of Sec. 2.1, reduced form with 2P
// interface rows):
//  Stage A, per partition with local rows j = 0..m-1 and neighbours x_{-1}
//  (end of the previous partition) and x_m (start of the next):
//    row 0 is normalised and set aside:  x_0 + a^_0 x_{-1} + c^_0 x_1 = d^_0;
//    rows j >= 1 are eliminated keeping x_0 as a parameter:
//      x_j + a^_j x_0 + c^_j x_{j+1} = d^_j,
//      j = 1: (a^, c^, d^) = (a, c, d)/b;   j >= 2: r = 1/(b_j - a_j c^_{j-1}),
//      a^_j = -r a_j a^_{j-1},  c^_j = r c_j,  d^_j = r (d_j - a_j d^_{j-1}).
//    Row m-1 is the partition's "last" interface equation.  Expressing x_1
//    through x_0 and x_{m-1} (back recurrence, accumulated forward with
//    running products pi_j = prod_{i<j} (-c^_i)) and substituting into row 0
//    gives the "first" interface equation.  Both have unit diagonal.
//  Stage B: the 2P interface rows of a system form a tridiagonal system
//    (first/last rows of partition p are rows 2p and 2p+1), solved in FP64
//    by parallel cyclic reduction: log2(2P) steps, each eliminating the
//    couplings at distance h and renormalising the diagonal to one.
//  Stage C: x_{m-1}, x_0 are interface unknowns; the interior follows from
//    x_j = d^_j - a^_j x_0 - c^_j x_{j+1}, j = m-2 .. 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdma_internal.h"

namespace tdma {
namespace dev {

template <typename T>
__device__ __forceinline__ bool bad_pivot(T v) {
    // zero, NaN or infinite pivot (NaN fails both comparisons)
    const T av = v < T(0) ? -v : v;
    return !(av > T(0) && av < T(__builtin_huge_val()));
}

// Reciprocal from the hardware estimate y plus a refinement of its residual
// e = 1 - x y.  FP64: one second-order step y (1 + e + e^2) (the geometric
// series of 1/(1 - e) truncated after e^2): the estimate is good to about
// 2^-24 (measured 4.6e-8 relative on this GPU), so the step leaves an error
// of order e^3, below half an ulp; measured bit-identical to two Newton steps
// on 4M samples over 600 binades, with three dependent operations after the
// estimate instead of four.  FP32: one Newton step y + y e.  About one ulp
// either way (the compiler's IEEE division adds scaling and fix-up steps these
// well-scaled pivots do not need).  A zero pivot gives a non-finite result and
// is flagged separately.
__device__ __forceinline__ double recip(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, __builtin_fma(e, e, e), y);
}

__device__ __forceinline__ float recip(float x) {
    const float y = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(y, e, y);
}

struct LaneSys {
    int64_t base;
    int64_t nrows;
    int64_t id;
    bool valid;
};

// Tile taken by block b of nb when the hardware hands consecutive block
// indices to the device's 8 XCDs in turn: the blocks of one XCD take
// consecutive tiles, so neighbouring tiles (which may share 128-byte lines
// when a tile row is narrower than a line) run at the same time under one
// L2.  A bijection of [0, nb).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    constexpr int64_t kXcds = 8;
    const int64_t q = nb / kXcds, r = nb % kXcds;
    const int64_t x = b % kXcds, i = b / kXcds;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Systems covered by a launch: nsys, or the device-side count when given.
__device__ __forceinline__ int64_t launch_nsys(const SysMap &m) {
    if (!m.count) return m.nsys;
    const int64_t c = (int64_t)*m.count;
    return c < m.nsys ? c : m.nsys;
}

__device__ __forceinline__ LaneSys lane_system(const SysMap &m, int64_t k) {
    LaneSys r;
    r.valid = k < launch_nsys(m);
    const int64_t kk = r.valid ? k : 0;
    const int64_t id = m.sys_list ? (int64_t)m.sys_list[kk] : kk;
    r.id = id;
    if (m.offsets) {
        r.base = m.offsets[id];
        r.nrows = m.offsets[id + 1] - r.base;
    } else {
        const int64_t s1 = id / m.nsys0;
        const int64_t s0 = id - s1 * m.nsys0;
        r.base = s0 * m.sys_stride0 + s1 * m.sys_stride1;
        r.nrows = m.n;
    }
    if (!r.valid) r.nrows = 0;
    return r;
}

// LDS bytes of Stage B for S systems x P partitions: three arrays (a, c, d)
// of 2P rows per system plus one pad row (both PCR variants fit in this).
__host__ __device__ constexpr size_t pcr_lds_bytes(int S, int P) {
    return (size_t)3 * S * (2 * P + 1) * sizeof(double);
}

// Interface rows of one partition (unit diagonal): first row couples
// (X_{2p-1}, X_{2p}, X_{2p+1}), last row couples (X_{2p}, X_{2p+1}, X_{2p+2}).
struct Iface {
    double fa, fc, fd;
    double la, lc, ld;
};

// Stage A on M register rows.  On return av/cv/dv hold a^, c^, d^ for rows
// 1..M-1 (row 0 values are folded into the first interface row).
template <typename T, int M>
__device__ __forceinline__ Iface reduce_partition(T (&av)[M], const T (&bv)[M], T (&cv)[M],
                                                  T (&dv)[M], bool &bad) {
    static_assert(M >= 2, "a partition needs at least two rows");
    T piv = bv[0];
    bad |= bad_pivot(piv);
    T ib = recip(piv);
    const T a0 = av[0] * ib, c0 = cv[0] * ib, d0 = dv[0] * ib;
    piv = bv[1];
    bad |= bad_pivot(piv);
    ib = recip(piv);
    av[1] *= ib;
    cv[1] *= ib;
    dv[1] *= ib;
#pragma unroll
    for (int j = 2; j < M; ++j) {
        piv = bv[j] - av[j] * cv[j - 1];
        bad |= bad_pivot(piv);
        ib = recip(piv);
        const T ra = av[j] * ib;
        dv[j] = (dv[j] - av[j] * dv[j - 1]) * ib;
        cv[j] = cv[j] * ib;
        av[j] = -ra * av[j - 1];
    }
    // x_1 = dt1 - at1 x_0 - ct1 x_{M-1}:  dt1 = sum_j pi_j d^_j, at1 = sum_j pi_j a^_j,
    // ct1 = -pi_{M-1}, with pi_1 = 1, pi_{j+1} = -c^_j pi_j, j = 1..M-2.
    T pi = T(1), dt1 = T(0), at1 = T(0);
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        dt1 += pi * dv[j];
        at1 += pi * av[j];
        pi = -cv[j] * pi;
    }
    const T ct1 = -pi;
    Iface f;
    const double den = 1.0 - (double)c0 * (double)at1;
    bad |= bad_pivot(den);
    const double rho = recip(den);
    f.fa = rho * (double)a0;
    f.fc = -rho * (double)c0 * (double)ct1;
    f.fd = rho * ((double)d0 - (double)c0 * (double)dt1);
    f.la = (double)av[M - 1];
    f.lc = (double)cv[M - 1];
    f.ld = (double)dv[M - 1];
    return f;
}

// Stage C on M register rows: dv becomes x.
template <typename T, int M>
__device__ __forceinline__ void substitute_partition(const T (&av)[M], const T (&cv)[M], T (&dv)[M],
                                                     double x_first, double x_last) {
    const T xf = (T)x_first;
    dv[M - 1] = (T)x_last;
#pragma unroll
    for (int j = M - 2; j >= 1; --j) dv[j] = dv[j] - av[j] * xf - cv[j] * dv[j + 1];
    dv[0] = xf;
}

// Stage A with the coefficient rows read from LDS (a shared operator): CA,
// CB, CC point at the partition's first row of the tile's a, b and c rows;
// `sh` is added to the diagonal of the first rows_here rows (a per-system
// shift; the rows past the system are identity rows).  On return ah, ch and
// dv hold a^, c^ and d^ of rows 1..M-1, as reduce_partition leaves them, so
// that substitute_partition(ah, ch, dv, ...) finishes the partition; only
// three values per row stay in registers.
template <typename T, int M, bool SHIFT>
__device__ __forceinline__ Iface reduce_partition_rows(const T *CA, const T *CB, const T *CC,
                                                       T sh, int rows_here, T (&ah)[M], T (&ch)[M],
                                                       T (&dv)[M], bool &bad) {
    static_assert(M >= 2, "a partition needs at least two rows");
    auto bj = [&](int j) {
        T b = CB[j];
        if constexpr (SHIFT) b += j < rows_here ? sh : T(0);
        return b;
    };
    T piv = bj(0);
    bad |= bad_pivot(piv);
    T ib = recip(piv);
    const T a0 = CA[0] * ib, c0 = CC[0] * ib, d0 = dv[0] * ib;
    piv = bj(1);
    bad |= bad_pivot(piv);
    ib = recip(piv);
    ah[1] = CA[1] * ib;
    ch[1] = CC[1] * ib;
    dv[1] *= ib;
#pragma unroll
    for (int j = 2; j < M; ++j) {
        const T aj = CA[j];
        piv = bj(j) - aj * ch[j - 1];
        bad |= bad_pivot(piv);
        ib = recip(piv);
        const T ra = aj * ib;
        dv[j] = (dv[j] - aj * dv[j - 1]) * ib;
        ch[j] = CC[j] * ib;
        ah[j] = -ra * ah[j - 1];
    }
    T pi = T(1), dt1 = T(0), at1 = T(0);
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        dt1 += pi * dv[j];
        at1 += pi * ah[j];
        pi = -ch[j] * pi;
    }
    const T ct1 = -pi;
    Iface f;
    const double den = 1.0 - (double)c0 * (double)at1;
    bad |= bad_pivot(den);
    const double rho = recip(den);
    f.fa = rho * (double)a0;
    f.fc = -rho * (double)c0 * (double)ct1;
    f.fd = rho * ((double)d0 - (double)c0 * (double)dt1);
    f.la = (double)ah[M - 1];
    f.lc = (double)ch[M - 1];
    f.ld = (double)dv[M - 1];
    return f;
}

// Stage B: PCR over the 2P interface rows of the S systems of a tile, in LDS.
// Row i of system s lives at i*S + s of each of the three arrays (unit
// diagonal kept implicit).  Lane (p, s) owns rows 2p and 2p+1; every thread
// of the block must call this.  Returns X_{2p} and X_{2p+1}.
__device__ __forceinline__ void pcr_interface(double *lds, int S, int s, int p, int P, Iface f,
                                              double &x_first, double &x_last, bool &bad) {
    const int R2 = 2 * P;
    double *ra = lds, *rc = lds + R2 * S, *rd = lds + 2 * R2 * S;
    const int i0 = 2 * p, i1 = 2 * p + 1;
    double a0 = f.fa, c0 = f.fc, d0 = f.fd, a1 = f.la, c1 = f.lc, d1 = f.ld;
    __syncthreads();
    ra[i0 * S + s] = a0; rc[i0 * S + s] = c0; rd[i0 * S + s] = d0;
    ra[i1 * S + s] = a1; rc[i1 * S + s] = c1; rd[i1 * S + s] = d1;
    __syncthreads();
    for (int h = 1; h < R2; h <<= 1) {
        double am0 = 0, cm0 = 0, dm0 = 0, ap0 = 0, cp0 = 0, dp0 = 0;
        double am1 = 0, cm1 = 0, dm1 = 0, ap1 = 0, cp1 = 0, dp1 = 0;
        if (i0 - h >= 0) { const int q = (i0 - h) * S + s; am0 = ra[q]; cm0 = rc[q]; dm0 = rd[q]; }
        if (i0 + h < R2) { const int q = (i0 + h) * S + s; ap0 = ra[q]; cp0 = rc[q]; dp0 = rd[q]; }
        if (i1 - h >= 0) { const int q = (i1 - h) * S + s; am1 = ra[q]; cm1 = rc[q]; dm1 = rd[q]; }
        if (i1 + h < R2) { const int q = (i1 + h) * S + s; ap1 = ra[q]; cp1 = rc[q]; dp1 = rd[q]; }
        {
            const double beta = 1.0 - a0 * cm0 - c0 * ap0;
            bad |= bad_pivot(beta);
            const double ib = recip(beta);
            const double na = -a0 * am0, nc = -c0 * cp0, nd = d0 - a0 * dm0 - c0 * dp0;
            a0 = na * ib; c0 = nc * ib; d0 = nd * ib;
        }
        {
            const double beta = 1.0 - a1 * cm1 - c1 * ap1;
            bad |= bad_pivot(beta);
            const double ib = recip(beta);
            const double na = -a1 * am1, nc = -c1 * cp1, nd = d1 - a1 * dm1 - c1 * dp1;
            a1 = na * ib; c1 = nc * ib; d1 = nd * ib;
        }
        if (2 * h < R2) {
            __syncthreads();
            ra[i0 * S + s] = a0; rc[i0 * S + s] = c0; rd[i0 * S + s] = d0;
            ra[i1 * S + s] = a1; rc[i1 * S + s] = c1; rd[i1 * S + s] = d1;
            __syncthreads();
        }
    }
    x_first = d0;
    x_last = d1;
}

// One PCR elimination step on a unit-diagonal row (a, c, d) with its
// neighbours at distance h below (al, cl, dl) and above (au, cu, du); the
// result is renormalised to unit diagonal.  Missing neighbours are zero rows.
__device__ __forceinline__ void pcr_row(double &a, double &c, double &d, double al, double cl,
                                        double dl, double au, double cu, double du, bool &bad) {
    const double beta = 1.0 - a * cl - c * au;
    bad |= bad_pivot(beta);
    const double ib = recip(beta);
    const double na = -a * al, nc = -c * cu, nd = d - a * dl - c * du;
    a = na * ib;
    c = nc * ib;
    d = nd * ib;
}

// Stage B inside wavefronts: the tile's interface rows go through LDS once,
// then P consecutive lanes (P a power of two <= 64, so one system never spans
// two wavefronts) each hold two rows of one system and run the PCR steps with
// cross-lane shuffles; the solution goes back through LDS.  Two barriers in
// total instead of two per step.
__device__ __forceinline__ void pcr_interface_wave(double *lds, int S, int s, int p, int P,
                                                   int P_log2, Iface f, double &x_first,
                                                   double &x_last, bool &bad) {
    const int R2 = 2 * P;
    const int pitch = R2 + 1;           // odd pitch: consecutive systems hit different banks
    const int nsys_rows = S * pitch;
    double *ra = lds, *rc = lds + nsys_rows, *rd = lds + 2 * nsys_rows;
    __syncthreads();
    {
        const int q = s * pitch + 2 * p;
        ra[q] = f.fa; rc[q] = f.fc; rd[q] = f.fd;
        ra[q + 1] = f.la; rc[q + 1] = f.lc; rd[q + 1] = f.ld;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int s2 = t >> P_log2;
    const int p2 = t & (P - 1);
    const int q2 = s2 * pitch + 2 * p2;
    double a0 = ra[q2], c0 = rc[q2], d0 = rd[q2];
    double a1 = ra[q2 + 1], c1 = rc[q2 + 1], d1 = rd[q2 + 1];
    const int lane = t & 63;
    {
        // h = 1: row 2p2 meets row 2p2-1 (lane-1) and its own row 2p2+1;
        // row 2p2+1 meets its own row 2p2 and row 2p2+2 (lane+1).
        const bool has_lo = p2 > 0, has_hi = p2 < P - 1;
        const int lo = has_lo ? lane - 1 : lane, hi = has_hi ? lane + 1 : lane;
        double am = __shfl(a1, lo), cm = __shfl(c1, lo), dm = __shfl(d1, lo);
        double ap = __shfl(a0, hi), cp = __shfl(c0, hi), dp = __shfl(d0, hi);
        if (!has_lo) { am = 0.0; cm = 0.0; dm = 0.0; }
        if (!has_hi) { ap = 0.0; cp = 0.0; dp = 0.0; }
        const double oa0 = a0, oc0 = c0, od0 = d0;
        pcr_row(a0, c0, d0, am, cm, dm, a1, c1, d1, bad);
        pcr_row(a1, c1, d1, oa0, oc0, od0, ap, cp, dp, bad);
    }
    for (int h = 2; h < R2; h <<= 1) {
        const int dl = h >> 1;          // rows 2p2+e +- h live in lanes p2 +- h/2
        const bool has_lo = p2 >= dl, has_hi = p2 + dl < P;
        const int lo = has_lo ? lane - dl : lane, hi = has_hi ? lane + dl : lane;
        double la0 = __shfl(a0, lo), lc0 = __shfl(c0, lo), ld0 = __shfl(d0, lo);
        double la1 = __shfl(a1, lo), lc1 = __shfl(c1, lo), ld1 = __shfl(d1, lo);
        double ua0 = __shfl(a0, hi), uc0 = __shfl(c0, hi), ud0 = __shfl(d0, hi);
        double ua1 = __shfl(a1, hi), uc1 = __shfl(c1, hi), ud1 = __shfl(d1, hi);
        if (!has_lo) { la0 = lc0 = ld0 = la1 = lc1 = ld1 = 0.0; }
        if (!has_hi) { ua0 = uc0 = ud0 = ua1 = uc1 = ud1 = 0.0; }
        pcr_row(a0, c0, d0, la0, lc0, ld0, ua0, uc0, ud0, bad);
        pcr_row(a1, c1, d1, la1, lc1, ld1, ua1, uc1, ud1, bad);
    }
    // each lane overwrites only its own two slots: no barrier needed before
    rd[q2] = d0;
    rd[q2 + 1] = d1;
    __syncthreads();
    x_first = rd[s * pitch + 2 * p];
    x_last = rd[s * pitch + 2 * p + 1];
}

template <typename T>
struct Ident {
    static constexpr T a = T(0), b = T(1), c = T(0), d = T(0);
};

// Per-tile system table for the LDS-staged (contiguous-row) path.
struct TileSysLds {
    int64_t base;
    int64_t nrows;
};

// A tile's rows of a shared operator (three coefficient arrays of length n),
// copied to LDS in two steps.  rows_prefetch loads rows tid + i*blockDim
// (i < CR) into registers, before the tile's right-hand sides are loaded:
// load counters retire in issue order, so whatever waits on these rows then
// leaves the right-hand sides in flight.  rows_commit writes them (and loads
// any rows beyond CR per thread) as CO[0..R) = a, CO[R..2R) = b,
// CO[2R..3R) = c with the corners removed and identity rows past n, then
// waits at a barrier.  Every thread of the block calls both.
template <int CR>
struct RowRegs {
    double a[CR], b[CR], c[CR];
};

template <typename T, int CR>
__device__ __forceinline__ void rows_prefetch(const Coef &coef, int64_t n, RowRegs<CR> &rr) {
    const T *A = (const T *)coef.a, *B = (const T *)coef.b, *C = (const T *)coef.c;
#pragma unroll
    for (int i = 0; i < CR; ++i) {
        const int64_t r = threadIdx.x + (int64_t)i * blockDim.x;
        const int64_t rc = r < n ? r : n - 1;
        rr.a[i] = (double)A[rc];
        rr.b[i] = (double)B[rc];
        rr.c[i] = (double)C[rc];
    }
}

template <typename T, int CR, typename LT = double>
__device__ __forceinline__ void rows_commit(LT *CO, const Coef &coef, int64_t n, int R,
                                            const RowRegs<CR> &rr) {
    const int nth = (int)blockDim.x;
#pragma unroll
    for (int i = 0; i < CR; ++i) {
        const int r = (int)threadIdx.x + i * nth;
        if (r < R) {
            const bool in = r < n;
            CO[r] = (LT)(in && r > 0 ? rr.a[i] : 0.0);
            CO[R + r] = (LT)(in ? rr.b[i] : 1.0);
            CO[2 * R + r] = (LT)(in && r < n - 1 ? rr.c[i] : 0.0);
        }
    }
    const T *A = (const T *)coef.a, *B = (const T *)coef.b, *C = (const T *)coef.c;
    for (int r = (int)threadIdx.x + CR * nth; r < R; r += nth) {
        const bool in = r < n;
        CO[r] = (LT)(in && r > 0 ? (double)A[r] : 0.0);
        CO[R + r] = (LT)(in ? (double)B[r] : 1.0);
        CO[2 * R + r] = (LT)(in && r < n - 1 ? (double)C[r] : 0.0);
    }
    __syncthreads();
}

// The thread index as a value the compiler cannot see through: index math
// derived from it is then recomputed in each staging call instead of being
// kept live in registers from one call to the next.
__device__ __forceinline__ int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Tile element e (0 <= e < S*R, rows of a system contiguous) as (system,
// row): float reciprocal of R with a one-step correction.
__device__ __forceinline__ void split_elem(int e, int R, float invR, int &se, int &re) {
    se = (int)(((float)e + 0.5f) * invR);
    re = e - se * R;
    if (re < 0) { --se; re += R; } else if (re >= R) { ++se; re -= R; }
}

// Cooperative coalesced copy of one tile array (S systems x R rows, rows
// contiguous in memory) into the lanes' registers, in two steps so that the
// loads of several arrays can all be in flight at once:
//   stage_load issues this thread's M loads (elements e = tid + i*blockDim)
//     with no branches: rows past a system's end read its last row and lanes
//     past the last system read the array's start (both replaced in stage_put);
//   stage_put writes them to LDS (identity value in the padding) and gives
//     each lane its M rows.
// The tile's S*P lanes call both (blockDim.x * M == S * R), after a barrier
// that makes the tile's system table visible.
template <typename T, int M>
__device__ __forceinline__ void stage_load(const TileSysLds *tsys, const T *src, int S, int R,
                                           float invR, T (&v)[M]) {
    const int tot = S * R;
    const int tid = opaque_tid();
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e0 = tid + i * (int)blockDim.x;
        const int e = e0 < tot ? e0 : tot - 1;
        int se, re;
        split_elem(e, R, invR, se, re);
        const int64_t nr = tsys[se].nrows;
        const int64_t rr = re < nr ? re : (nr > 0 ? nr - 1 : 0);
        v[i] = src[(nr > 0 ? tsys[se].base : 0) + rr];
    }
}

template <typename T, int M>
__device__ __forceinline__ void stage_put(T *stg, const TileSysLds *tsys, T ident, int S, int R,
                                          int pitch, float invR, int s, int r0, const T (&v)[M],
                                          T (&dst)[M]) {
    const int tot = S * R;
    __syncthreads();   // the staging buffer is free
    const int tid = opaque_tid();
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e = tid + i * (int)blockDim.x;
        if (e < tot) {
            int se, re;
            split_elem(e, R, invR, se, re);
            stg[se * pitch + re] = re < tsys[se].nrows ? v[i] : ident;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M; ++j) dst[j] = stg[s * pitch + r0 + j];
}

// One array in one pass (barrier for the system table included), with K of
// a thread's loads in flight at a time: each group of K goes to LDS before
// the next is issued, which bounds the registers that hold their addresses.
template <typename T, int M, int K = 4>
__device__ __forceinline__ void stage_in(T *stg, const TileSysLds *tsys, const T *src, T ident,
                                         int S, int R, int pitch, float invR, int s, int r0,
                                         T (&dst)[M]) {
    static_assert(M % K == 0, "K must divide M");
    const int tot = S * R;
    __syncthreads();
    const int tid = opaque_tid();
#pragma unroll
    for (int c = 0; c < M; c += K) {
        T v[K];
        int se[K], re[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e0 = tid + (c + k) * (int)blockDim.x;
            split_elem(e0 < tot ? e0 : tot - 1, R, invR, se[k], re[k]);
            const int64_t nr = tsys[se[k]].nrows;
            const int64_t rr = re[k] < nr ? re[k] : (nr > 0 ? nr - 1 : 0);
            v[k] = src[(nr > 0 ? tsys[se[k]].base : 0) + rr];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e0 = tid + (c + k) * (int)blockDim.x;
            if (e0 < tot) stg[se[k] * pitch + re[k]] = re[k] < tsys[se[k]].nrows ? v[k] : ident;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M; ++j) dst[j] = stg[s * pitch + r0 + j];
}

template <typename T, int M>
__device__ __forceinline__ void stage_out(T *stg, const TileSysLds *tsys, T *dst_g, int S, int R,
                                          int pitch, float invR, int s, int r0, const T (&src)[M]) {
    const int nthr = blockDim.x;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M; ++j) stg[s * pitch + r0 + j] = src[j];
    __syncthreads();
    for (int e = threadIdx.x; e < S * R; e += nthr) {
        int se, re;
        split_elem(e, R, invR, se, re);
        if (re < tsys[se].nrows) dst_g[tsys[se].base + re] = stg[se * pitch + re];
    }
}

// The same copies with each lane's M rows at a stride of M+1 in LDS (row re
// of a system at slot re + re/M, systems `pitch` = P*(M+1)+1 slots apart):
// the lanes of a wavefront, which hold consecutive partitions of a system,
// then read and write their rows at an odd stride of 8-byte words, without
// the bank conflicts of a stride of M rows.
template <int M>
__device__ __forceinline__ int sw_slot(int re) { return re + re / M; }

template <typename T, int M, int K = 4>
__device__ __forceinline__ void stage_in_sw(T *stg, const TileSysLds *tsys, const T *src, T ident,
                                            int S, int R, int pitch, float invR, int s, int p,
                                            T (&dst)[M]) {
    static_assert(M % K == 0, "K must divide M");
    const int tot = S * R;
    __syncthreads();
    const int tid = opaque_tid();
#pragma unroll
    for (int c = 0; c < M; c += K) {
        T v[K];
        int se[K], re[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e0 = tid + (c + k) * (int)blockDim.x;
            split_elem(e0 < tot ? e0 : tot - 1, R, invR, se[k], re[k]);
            const int64_t nr = tsys[se[k]].nrows;
            const int64_t rr = re[k] < nr ? re[k] : (nr > 0 ? nr - 1 : 0);
            v[k] = src[(nr > 0 ? tsys[se[k]].base : 0) + rr];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e0 = tid + (c + k) * (int)blockDim.x;
            if (e0 < tot) stg[se[k] * pitch + sw_slot<M>(re[k])] = re[k] < tsys[se[k]].nrows ? v[k] : ident;
        }
    }
    __syncthreads();
    const int q = s * pitch + p * (M + 1);
#pragma unroll
    for (int j = 0; j < M; ++j) dst[j] = stg[q + j];
}

// All four arrays of a per-row tile (a, b, c, d; rows contiguous) at once:
// every thread issues its M loads of each array (elements tid + i*blockDim,
// the same offsets for the four), so the four arrays' loads are in flight
// together, then the arrays pass through the staging buffer one after the
// other in place, each lane taking its own rows (identity values past a
// system's end).  blockDim.x * M == S * R.
template <typename T, int M>
__device__ __forceinline__ void stage_in4_sw(T *stg, const TileSysLds *tsys, const T *A, const T *B,
                                             const T *C, const T *D, int S, int R, int pitch,
                                             float invR, int s, int p, T (&av)[M], T (&bv)[M],
                                             T (&cv)[M], T (&dv)[M]) {
    __syncthreads();
    const int tot = S * R;
    const int tid = opaque_tid();
    int slot[M];
    bool in[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e0 = tid + i * (int)blockDim.x;
        const int e = e0 < tot ? e0 : tot - 1;
        int se, re;
        split_elem(e, R, invR, se, re);
        const int64_t nr = tsys[se].nrows;
        const int64_t rr = re < nr ? re : (nr > 0 ? nr - 1 : 0);
        const int64_t o = (nr > 0 ? tsys[se].base : 0) + rr;
        av[i] = A[o];
        bv[i] = B[o];
        cv[i] = C[o];
        dv[i] = D[o];
        slot[i] = se * pitch + sw_slot<M>(re);
        in[i] = re < nr;
    }
    const int q = s * pitch + p * (M + 1);
    auto put = [&](T (&v)[M], T ident) {
#pragma unroll
        for (int i = 0; i < M; ++i) stg[slot[i]] = in[i] ? v[i] : ident;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < M; ++j) v[j] = stg[q + j];
        __syncthreads();
    };
    put(dv, Ident<T>::d);
    put(av, Ident<T>::a);
    put(bv, Ident<T>::b);
    put(cv, Ident<T>::c);
}

template <typename T, int M>
__device__ __forceinline__ void stage_out_sw(T *stg, const TileSysLds *tsys, T *dst_g, int S, int R,
                                             int pitch, float invR, int s, int p, const T (&src)[M]) {
    const int nthr = blockDim.x;
    __syncthreads();
    const int q = s * pitch + p * (M + 1);
#pragma unroll
    for (int j = 0; j < M; ++j) stg[q + j] = src[j];
    __syncthreads();
    for (int e = threadIdx.x; e < S * R; e += nthr) {
        int se, re;
        split_elem(e, R, invR, se, re);
        if (re < tsys[se].nrows) dst_g[tsys[se].base + re] = stg[se * pitch + sw_slot<M>(re)];
    }
}

}  // namespace dev
}  // namespace tdma
