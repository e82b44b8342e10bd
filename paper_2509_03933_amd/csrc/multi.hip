// Several right-hand sides per system over one shared operator (a shared
// coefficient table, optionally with a per-system diagonal shift).  The
// paper's Poisson lines are the motivating case (Sec. 5.2 and 8.1): after the
// Fourier transform in x and y every z-line has a real operator and a complex
// right-hand side, i.e. two real right-hand sides (real and imaginary parts,
// interleaved in memory).
//
// The partition sweep of Stage A splits into a coefficient recurrence
// (pivots, a^, c^: one reciprocal per row) that depends only on the operator,
// and a right-hand-side recurrence (d^) that is linear in d.  A lane runs the
// first once for its M rows and the second once per right-hand side, so the
// registers per row are 2 + NR values instead of 3 * NR and the reciprocals
// are shared.  Stage B likewise eliminates the interface operator once and
// carries NR right-hand sides through every PCR step; Stage C substitutes
// each right-hand side with the shared a^, c^.
#include <type_traits>

#include "tile.hip.h"

namespace tdma {

namespace {

using dev::LaneSys;

template <int NR>
struct IfaceN {
    double fa, fc, la, lc;      // shared by every right-hand side
    double fd[NR], ld[NR];
};

// Stage A for NR right-hand sides with the operator's rows in LDS (CA, CB,
// CC: the partition's first row of the tile's a, b, c rows; rows past the
// system are identity rows).  Same recurrences as reduce_partition_rows, the
// d^ recurrence and the interface right-hand sides once per right-hand side.
template <typename T, int M, int NR, bool SHIFT>
__device__ __forceinline__ IfaceN<NR> reduce_rows_multi(const T *CA, const T *CB, const T *CC,
                                                        T sh, int rows_here, T (&ah)[M],
                                                        T (&ch)[M], T (&dv)[NR][M], bool &bad) {
    static_assert(M >= 2, "a partition needs at least two rows");
    auto bj = [&](int j) {
        T b = CB[j];
        if constexpr (SHIFT) b += j < rows_here ? sh : T(0);
        return b;
    };
    T piv = bj(0);
    bad |= dev::bad_pivot(piv);
    T ib = dev::recip(piv);
    const T a0 = CA[0] * ib, c0 = CC[0] * ib;
    T d0[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) d0[r] = dv[r][0] * ib;
    piv = bj(1);
    bad |= dev::bad_pivot(piv);
    ib = dev::recip(piv);
    ah[1] = CA[1] * ib;
    ch[1] = CC[1] * ib;
#pragma unroll
    for (int r = 0; r < NR; ++r) dv[r][1] *= ib;
#pragma unroll
    for (int j = 2; j < M; ++j) {
        const T aj = CA[j];
        piv = bj(j) - aj * ch[j - 1];
        bad |= dev::bad_pivot(piv);
        ib = dev::recip(piv);
        const T ra = aj * ib;
#pragma unroll
        for (int r = 0; r < NR; ++r) dv[r][j] = (dv[r][j] - aj * dv[r][j - 1]) * ib;
        ch[j] = CC[j] * ib;
        ah[j] = -ra * ah[j - 1];
    }
    // x_1 = dt1 - at1 x_0 - ct1 x_{M-1} with the running products pi_j
    T pi = T(1), at1 = T(0);
    T dt1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dt1[r] = T(0);
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) dt1[r] += pi * dv[r][j];
        at1 += pi * ah[j];
        pi = -ch[j] * pi;
    }
    const T ct1 = -pi;
    IfaceN<NR> f;
    const double den = 1.0 - (double)c0 * (double)at1;
    bad |= dev::bad_pivot(den);
    const double rho = dev::recip(den);
    f.fa = rho * (double)a0;
    f.fc = -rho * (double)c0 * (double)ct1;
    f.la = (double)ah[M - 1];
    f.lc = (double)ch[M - 1];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        f.fd[r] = rho * ((double)d0[r] - (double)c0 * (double)dt1[r]);
        f.ld[r] = (double)dv[r][M - 1];
    }
    return f;
}

// One PCR step on a unit-diagonal row (a, c) with NR right-hand sides d,
// neighbours at distance h below (al, cl, dl) and above (au, cu, du).
template <int NR>
__device__ __forceinline__ void pcr_row_multi(double &a, double &c, double (&d)[NR], double al,
                                              double cl, const double (&dl)[NR], double au,
                                              double cu, const double (&du)[NR], bool &bad) {
    const double beta = 1.0 - a * cl - c * au;
    bad |= dev::bad_pivot(beta);
    const double ib = dev::recip(beta);
#pragma unroll
    for (int r = 0; r < NR; ++r) d[r] = (d[r] - a * dl[r] - c * du[r]) * ib;
    const double na = -a * al, nc = -c * cu;
    a = na * ib;
    c = nc * ib;
}

// Stage B for NR right-hand sides inside wavefronts (P a power of two <= 64):
// the interface rows go through LDS once, P consecutive lanes each hold rows
// 2p and 2p+1 of one system and run the PCR steps with cross-lane shuffles,
// and the solution goes back through LDS.  LDS: (2 + NR) arrays of S systems
// x (2P + 1) doubles.  Every thread of the block calls it.
template <int NR>
__device__ __forceinline__ void pcr_wave_multi(double *lds, int S, int s, int p, int P,
                                               int P_log2, const IfaceN<NR> &f,
                                               double (&x_first)[NR], double (&x_last)[NR],
                                               bool &bad) {
    const int pitch = 2 * P + 1;
    const int rows = S * pitch;
    double *ra = lds, *rc = lds + rows, *rd = lds + 2 * rows;
    __syncthreads();   // every lane is done with what this LDS held before
    {
        const int q = s * pitch + 2 * p;
        ra[q] = f.fa; rc[q] = f.fc;
        ra[q + 1] = f.la; rc[q + 1] = f.lc;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            rd[r * rows + q] = f.fd[r];
            rd[r * rows + q + 1] = f.ld[r];
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int s2 = t >> P_log2;
    const int p2 = t & (P - 1);
    const int q2 = s2 * pitch + 2 * p2;
    double a0 = ra[q2], c0 = rc[q2], a1 = ra[q2 + 1], c1 = rc[q2 + 1];
    double d0[NR], d1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        d0[r] = rd[r * rows + q2];
        d1[r] = rd[r * rows + q2 + 1];
    }
    const int lane = t & 63;
    {
        // h = 1: row 2p2 meets row 2p2-1 (last row of lane-1) and its own row
        // 2p2+1; row 2p2+1 meets its own row 2p2 and row 2p2+2 (lane+1)
        const bool has_lo = p2 > 0, has_hi = p2 < P - 1;
        const int lo = has_lo ? lane - 1 : lane, hi = has_hi ? lane + 1 : lane;
        double am = __shfl(a1, lo), cm = __shfl(c1, lo);
        double ap = __shfl(a0, hi), cp = __shfl(c0, hi);
        double dm[NR], dp[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            dm[r] = __shfl(d1[r], lo);
            dp[r] = __shfl(d0[r], hi);
            if (!has_lo) dm[r] = 0.0;
            if (!has_hi) dp[r] = 0.0;
        }
        if (!has_lo) { am = 0.0; cm = 0.0; }
        if (!has_hi) { ap = 0.0; cp = 0.0; }
        const double oa0 = a0, oc0 = c0;
        double od0[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) od0[r] = d0[r];
        pcr_row_multi<NR>(a0, c0, d0, am, cm, dm, a1, c1, d1, bad);
        pcr_row_multi<NR>(a1, c1, d1, oa0, oc0, od0, ap, cp, dp, bad);
    }
    for (int h = 2; h < 2 * P; h <<= 1) {
        const int dl = h >> 1;          // rows 2p2+e +- h live in lanes p2 +- h/2
        const bool has_lo = p2 >= dl, has_hi = p2 + dl < P;
        const int lo = has_lo ? lane - dl : lane, hi = has_hi ? lane + dl : lane;
        double la0 = __shfl(a0, lo), lc0 = __shfl(c0, lo), la1 = __shfl(a1, lo), lc1 = __shfl(c1, lo);
        double ua0 = __shfl(a0, hi), uc0 = __shfl(c0, hi), ua1 = __shfl(a1, hi), uc1 = __shfl(c1, hi);
        double ld0[NR], ld1[NR], ud0[NR], ud1[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            ld0[r] = __shfl(d0[r], lo); ld1[r] = __shfl(d1[r], lo);
            ud0[r] = __shfl(d0[r], hi); ud1[r] = __shfl(d1[r], hi);
            if (!has_lo) { ld0[r] = 0.0; ld1[r] = 0.0; }
            if (!has_hi) { ud0[r] = 0.0; ud1[r] = 0.0; }
        }
        if (!has_lo) { la0 = lc0 = la1 = lc1 = 0.0; }
        if (!has_hi) { ua0 = uc0 = ua1 = uc1 = 0.0; }
        pcr_row_multi<NR>(a0, c0, d0, la0, lc0, ld0, ua0, uc0, ud0, bad);
        pcr_row_multi<NR>(a1, c1, d1, la1, lc1, ld1, ua1, uc1, ud1, bad);
    }
    // each lane overwrites only its own two slots: no barrier needed before
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        rd[r * rows + q2] = d0[r];
        rd[r * rows + q2 + 1] = d1[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        x_first[r] = rd[r * rows + s * pitch + 2 * p];
        x_last[r] = rd[r * rows + s * pitch + 2 * p + 1];
    }
}

// LDS of one tile: the operator's 3 x P*M rows (type T) during Stage A, then
// the Stage B exchange, which reuses the same bytes.
inline size_t multi_lds_bytes(size_t esz, int S, int P, int M, int NR) {
    const size_t pcr = (size_t)(2 + NR) * S * (2 * P + 1) * sizeof(double);
    const size_t co = 3 * (size_t)P * M * esz;
    return pcr > co ? pcr : co;
}

// One tile per block: systems k0 .. k0+S-1, S*P lanes, M rows per lane, NR
// right-hand sides rhs_stride elements apart.  VEC: NR == 2 with rhs_stride
// 1 and every element pair 2*sizeof(T)-aligned, each row's two right-hand
// sides moved as one vector.  Loads and stores carry the non-temporal hint
// (each element is touched once; 11.2 -> 10.8 ms on the 1024^3 complex
// lines).
// Tile order: with spread > 0, block b takes tile (b * spread) mod nblocks
// (spread coprime to nblocks: a bijection), so the blocks running at one
// time hold tiles scattered over the whole system range.  A tile's rows
// share one offset modulo the row stride; on long power-of-two strides
// (the 16 MB rows of 1024^2 complex modes) neighbouring tiles then fall on
// the same memory channels, scattered ones do not.  With spread == 0 the
// order is XCD-aware (dev::xcd_tile), for tile rows narrower than a line.
// x may alias d: a block reads all of its tile before it writes any of it.
template <typename T, int M, int NR, bool SHIFT, bool VEC>
__global__ void __launch_bounds__(512)
k_multi(SysMap map, Coef coef, const T *d, T *x, int64_t rhs_stride, int S_log2, int P_log2,
        int64_t spread, int *err) {
    static_assert(!VEC || NR == 2, "vector form moves two right-hand sides");
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int S = 1 << S_log2;
    const int P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int R = P * M;
    const int64_t nb = gridDim.x;
    const int64_t k0 = (spread > 0 ? ((int64_t)blockIdx.x * spread) % nb
                                    : dev::xcd_tile(blockIdx.x, nb)) << S_log2;
    const LaneSys sys = dev::lane_system(map, k0 + s);
    const int rows_here = (int)(sys.nrows - r0 < 0 ? 0 : (sys.nrows - r0 > M ? M : sys.nrows - r0));
    T *CO = reinterpret_cast<T *>(lds);

    // operator rows first, then the right-hand sides (in flight while the
    // rows go to LDS); branch-free: the row index stops at the system's last
    // row and a lane past the last system reads the array's start
    constexpr int CR = 2;
    dev::RowRegs<CR> rr;
    dev::rows_prefetch<T, CR>(coef, map.n, rr);
    __builtin_amdgcn_sched_barrier(0);
    T dv[NR][M];
    const int64_t rs = map.row_stride;
    const int64_t last = sys.nrows > 0 ? sys.nrows - 1 : 0;
    const int64_t first = r0 < last ? r0 : last;
    const int adv = (int)(last - first < M ? last - first : M);
    {
        int64_t idx = (sys.valid ? sys.base : 0) + first * rs;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if constexpr (VEC) {
                typedef T T2 __attribute__((ext_vector_type(2)));
                const T2 v = __builtin_nontemporal_load(reinterpret_cast<const T2 *>(d + idx));
                dv[0][j] = v.x;
                dv[1][j] = v.y;
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) dv[r][j] = __builtin_nontemporal_load(d + idx + r * rhs_stride);
            }
            idx += j < adv ? rs : 0;
        }
    }
    T sh = T(0);
    if constexpr (SHIFT) {
        sh = ((const T *)coef.shift)[sys.valid ? sys.id : 0];
        if (!sys.valid) sh = T(0);
    }
    dev::rows_commit<T, CR, T>(CO, coef, map.n, R, rr);
#pragma unroll
    for (int j = 0; j < M; ++j)
        if (j >= rows_here) {
#pragma unroll
            for (int r = 0; r < NR; ++r) dv[r][j] = T(0);
        }

    bool bad = false;
    T ah[M], ch[M];
    const IfaceN<NR> f = reduce_rows_multi<T, M, NR, SHIFT>(CO + r0, CO + R + r0, CO + 2 * R + r0,
                                                            sh, rows_here, ah, ch, dv, bad);
    double xf[NR], xl[NR];
    pcr_wave_multi<NR>(lds, S, s, p, P, P_log2, f, xf, xl, bad);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const T xfr = (T)xf[r];
        dv[r][M - 1] = (T)xl[r];
#pragma unroll
        for (int j = M - 2; j >= 1; --j) dv[r][j] = dv[r][j] - ah[j] * xfr - ch[j] * dv[r][j + 1];
        dv[r][0] = xfr;
    }

    const int64_t off0 = sys.base + (int64_t)r0 * rs;
#pragma unroll
    for (int j = 0; j < M; ++j)
        if (j < rows_here) {
            const int64_t idx = off0 + j * rs;
            if constexpr (VEC) {
                typedef T T2 __attribute__((ext_vector_type(2)));
                T2 v;
                v.x = dv[0][j];
                v.y = dv[1][j];
                __builtin_nontemporal_store(v, reinterpret_cast<T2 *>(x + idx));
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) __builtin_nontemporal_store(dv[r][j], x + idx + r * rhs_stride);
            }
        }
    if (bad && sys.valid) atomicOr(err, 1);
}

// A stride near nb / phi (the golden ratio) that is coprime to nb, so that
// b -> b * stride mod nb is a bijection whose consecutive values are spread
// evenly over [0, nb); 0 (no spreading) below 64 tiles.
int64_t spread_stride(int64_t nb) {
    if (nb < 64) return 0;
    int64_t k = (int64_t)((double)nb * 0.6180339887498949) | 1;
    auto gcd = [](int64_t a, int64_t b) {
        while (b) {
            const int64_t t = a % b;
            a = b;
            b = t;
        }
        return a;
    };
    while (gcd(k, nb) != 1) k += 2;
    return k;
}

template <typename T, int M, int NR, bool SHIFT, bool VEC>
hipError_t launch_t(const SysMap &map, const Coef &coef, const MultiShape &sh, int64_t rhs_stride,
                    const void *d, void *x, int *err, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    const size_t lds = multi_lds_bytes(sizeof(T), (int)S, 1 << sh.P_log2, M, NR);
    // full 128-byte tile rows: scattered tile order; narrower: XCD-aware
    const int64_t row_bytes = S * (int64_t)sizeof(T) * (VEC ? 2 : 1);
    const int64_t spread = row_bytes >= 128 ? spread_stride(blocks) : 0;
    hipLaunchKernelGGL((k_multi<T, M, NR, SHIFT, VEC>), dim3((unsigned)blocks),
                       dim3((unsigned)(S << sh.P_log2)), lds, st, map, coef, (const T *)d, (T *)x,
                       rhs_stride, sh.S_log2, sh.P_log2, spread, err);
    return hipGetLastError();
}

template <typename T, int M>
hipError_t launch_group(const SysMap &map, const Coef &coef, const MultiShape &sh, int nr,
                        bool vec, int64_t rhs_stride, const void *d, void *x, int *err,
                        hipStream_t st) {
    const bool shift = coef.shift != nullptr;
#define TDMA_MULTI(NR, SH, V)                                                                   \
    if (nr == NR && shift == SH && vec == V)                                                    \
        return launch_t<T, M, NR, SH, V>(map, coef, sh, rhs_stride, d, x, err, st);
    TDMA_MULTI(2, true, true)
    TDMA_MULTI(2, false, true)
    TDMA_MULTI(2, true, false)
    TDMA_MULTI(2, false, false)
    TDMA_MULTI(1, true, false)
    TDMA_MULTI(1, false, false)
#undef TDMA_MULTI
    return hipErrorInvalidValue;
}

}  // namespace

bool multi_shape(int dtype, int64_t n, int64_t nsys, MultiShape *out) {
    const int M = dtype == TDMA_F64 ? 16 : 32;
    int P_log2 = 0;
    while (((int64_t)M << P_log2) < n) ++P_log2;
    if (P_log2 > 6) return false;          // P <= 64: one system per wavefront in Stage B
    int S_log2 = 9 - P_log2;               // S * P = 512 lanes
    if (S_log2 > 5) S_log2 = 5;
    while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
    out->M = M;
    out->P_log2 = P_log2;
    out->S_log2 = S_log2;
    return true;
}

size_t multi_lds(int dtype, const MultiShape &sh, int nr) {
    return multi_lds_bytes(dtype == TDMA_F64 ? 8 : 4, 1 << sh.S_log2, 1 << sh.P_log2, sh.M, nr);
}

hipError_t launch_multi(int dtype, const SysMap &map, const Coef &coef, const MultiShape &sh,
                        int nrhs, int64_t rhs_stride, bool vec, const void *d, void *x, int *err,
                        hipStream_t st) {
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    // groups of two right-hand sides, then a single one when nrhs is odd
    for (int r = 0; r < nrhs;) {
        const int nr = nrhs - r >= 2 ? 2 : 1;
        const char *dg = (const char *)d + (size_t)r * rhs_stride * esz;
        char *xg = (char *)x + (size_t)r * rhs_stride * esz;
        const bool v = vec && nr == 2;
        hipError_t e;
        if (dtype == TDMA_F64 && sh.M == 16)
            e = launch_group<double, 16>(map, coef, sh, nr, v, rhs_stride, dg, xg, err, st);
        else if (dtype == TDMA_F32 && sh.M == 32)
            e = launch_group<float, 32>(map, coef, sh, nr, v, rhs_stride, dg, xg, err, st);
        else
            e = hipErrorInvalidValue;
        if (e != hipSuccess) return e;
        r += nr;
    }
    return hipSuccess;
}

}  // namespace tdma
