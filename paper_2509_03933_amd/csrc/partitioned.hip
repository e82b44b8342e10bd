// Staged divide-and-conquer solve: three kernels per batch of systems.
//
// Stage A (k_stage_a): one lane per (system, partition) streams the partition
//   once, carrying only O(1) state: the modified Thomas recurrences of
//   tile.hip.h and the running products that turn the back recurrence of the
//   row-1 spike into a forward sum.  It writes the partition's two
//   unit-diagonal interface equations (6 values) to the reduced buffer, and
//   the row factors d^, a^, c^ that Stage C needs to a workspace (never to x,
//   so inputs and outputs never alias inside a kernel and loads can run ahead).
// Stage B (k_stage_b): the 2P-row interface system of every system of the
//   batch, FP64; parallel cyclic reduction across P consecutive lanes with
//   wavefront shuffles (P a power of two <= 64), otherwise one lane per system
//   eliminating the 2P rows in sequence.
// Stage C (k_stage_c): one lane per (system, partition) walks the partition
//   backwards: x_{m-1} and x_0 are interface unknowns and
//   x_j = d^_j - a^_j x_0 - c^_j x_{j+1}.
//
// Partition p of a system of n rows has m_p = floor(n/P) + (p < n mod P) rows
// starting at p*floor(n/P) + min(p, n mod P).  Every system's arithmetic is
// independent of how systems are batched, so results are bit-identical for
// any batch size, stream count or schedule.
#include "tile.hip.h"
#include "partitioned.h"

namespace tdma {
namespace {

struct PartRange {
    int64_t start;
    int m;
};

__device__ __forceinline__ PartRange part_range(int64_t n, int P, int p) {
    const int64_t q = n / P, r = n % P;
    PartRange pr;
    pr.start = p * q + (p < r ? p : r);
    pr.m = (int)(q + (p < r ? 1 : 0));
    return pr;
}

// Reduced-buffer layout: value v (0..5 = first a, c, d, last a, c, d) of
// partition p of batch-local system k at ((v*P + p) * nb + k).
__device__ __forceinline__ size_t red_at(int v, int p, int64_t k, int P, int64_t nb) {
    return ((size_t)v * P + p) * nb + k;
}

template <typename T, bool LIKE_D, bool SHIFT, bool SHARED_FACTORS>
__global__ void __launch_bounds__(256)
k_stage_a(SysMap map, Coef coef, const T *__restrict__ d, T *__restrict__ ws_d,
          T *__restrict__ ws_a, T *__restrict__ ws_c, double *__restrict__ red, int64_t k_begin,
          int64_t nb, int P, int *err) {
    const int64_t kl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (kl >= nb) return;
    const dev::LaneSys sys = dev::lane_system(map, k_begin + kl);
    const int64_t n = map.n;
    const PartRange pr = part_range(n, P, p);
    const T *__restrict__ A = (const T *)coef.a;
    const T *__restrict__ B = (const T *)coef.b;
    const T *__restrict__ C = (const T *)coef.c;
    const int64_t rs = map.row_stride;
    T sh = T(0);
    if constexpr (SHIFT) sh = ((const T *)coef.shift)[sys.id];
    auto load = [&](int64_t r, T &a, T &b, T &c, T &dd) {
        const int64_t idx = sys.base + r * rs;
        dd = d[idx];
        if constexpr (LIKE_D) {
            a = A[idx]; b = B[idx]; c = C[idx];
        } else {
            a = A[r]; b = B[r]; c = C[r];
        }
        if constexpr (SHIFT) b += sh;
        if (r == 0) a = T(0);
        if (r == n - 1) c = T(0);
    };
    // factor storage: row r of batch-local system kl at r*nb + kl (coalesced)
    const bool store_factors = !SHARED_FACTORS || kl == 0;
    const int64_t fk = SHARED_FACTORS ? 0 : kl;
    const int64_t fstride = SHARED_FACTORS ? 1 : nb;
    bool bad = false;
    T a, b, c, dd;
    load(pr.start, a, b, c, dd);
    bad |= dev::bad_pivot(b);
    T ib = dev::recip(b);
    const T a0 = a * ib, c0 = c * ib, d0 = dd * ib;
    load(pr.start + 1, a, b, c, dd);
    bad |= dev::bad_pivot(b);
    ib = dev::recip(b);
    T ah = a * ib, ch = c * ib, dh = dd * ib;
    T pi = T(1), dt1 = T(0), at1 = T(0);
    const int m = pr.m;
#pragma unroll 4
    for (int j = 1; j < m - 1; ++j) {
        // row j is final: store it, fold it into the row-1 spike, then advance
        const int64_t r = pr.start + j;
        ws_d[r * nb + kl] = dh;
        if (store_factors) {
            ws_a[r * fstride + fk] = ah;
            ws_c[r * fstride + fk] = ch;
        }
        dt1 += pi * dh;
        at1 += pi * ah;
        pi = -ch * pi;
        load(r + 1, a, b, c, dd);
        const T piv = b - a * ch;
        bad |= dev::bad_pivot(piv);
        ib = dev::recip(piv);
        const T ra = a * ib;
        dh = (dd - a * dh) * ib;
        ch = c * ib;
        ah = -ra * ah;
    }
    const T ct1 = -pi;
    const double den = 1.0 - (double)c0 * (double)at1;
    bad |= dev::bad_pivot(den);
    const double rho = dev::recip(den);
    red[red_at(0, p, kl, P, nb)] = rho * (double)a0;
    red[red_at(1, p, kl, P, nb)] = -rho * (double)c0 * (double)ct1;
    red[red_at(2, p, kl, P, nb)] = rho * ((double)d0 - (double)c0 * (double)dt1);
    red[red_at(3, p, kl, P, nb)] = (double)ah;
    red[red_at(4, p, kl, P, nb)] = (double)ch;
    red[red_at(5, p, kl, P, nb)] = (double)dh;
    if (bad) atomicOr(err, 1);
}

// Stage B, PCR variant: P consecutive lanes per system (P power of two <= 64).
__global__ void __launch_bounds__(256)
k_stage_b_pcr(const double *red, double *X, int64_t nb, int P, int P_log2, int *err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kl = t >> P_log2;
    const int p = (int)(t & (P - 1));
    const bool valid = kl < nb;
    const int64_t kk = valid ? kl : 0;
    double a0 = red[red_at(0, p, kk, P, nb)], c0 = red[red_at(1, p, kk, P, nb)];
    double d0 = red[red_at(2, p, kk, P, nb)], a1 = red[red_at(3, p, kk, P, nb)];
    double c1 = red[red_at(4, p, kk, P, nb)], d1 = red[red_at(5, p, kk, P, nb)];
    const int lane = threadIdx.x & 63;
    bool bad = false;
    for (int h = 1; h < 2 * P; h <<= 1) {
        if (h == 1) {
            const bool has_lo = p > 0, has_hi = p < P - 1;
            const int lo = has_lo ? lane - 1 : lane, hi = has_hi ? lane + 1 : lane;
            double am = __shfl(a1, lo), cm = __shfl(c1, lo), dm = __shfl(d1, lo);
            double ap = __shfl(a0, hi), cp = __shfl(c0, hi), dp = __shfl(d0, hi);
            if (!has_lo) { am = 0.0; cm = 0.0; dm = 0.0; }
            if (!has_hi) { ap = 0.0; cp = 0.0; dp = 0.0; }
            const double oa0 = a0, oc0 = c0, od0 = d0;
            dev::pcr_row(a0, c0, d0, am, cm, dm, a1, c1, d1, bad);
            dev::pcr_row(a1, c1, d1, oa0, oc0, od0, ap, cp, dp, bad);
        } else {
            const int dl = h >> 1;
            const bool has_lo = p >= dl, has_hi = p + dl < P;
            const int lo = has_lo ? lane - dl : lane, hi = has_hi ? lane + dl : lane;
            double la0 = __shfl(a0, lo), lc0 = __shfl(c0, lo), ld0 = __shfl(d0, lo);
            double la1 = __shfl(a1, lo), lc1 = __shfl(c1, lo), ld1 = __shfl(d1, lo);
            double ua0 = __shfl(a0, hi), uc0 = __shfl(c0, hi), ud0 = __shfl(d0, hi);
            double ua1 = __shfl(a1, hi), uc1 = __shfl(c1, hi), ud1 = __shfl(d1, hi);
            if (!has_lo) { la0 = lc0 = ld0 = la1 = lc1 = ld1 = 0.0; }
            if (!has_hi) { ua0 = uc0 = ud0 = ua1 = uc1 = ud1 = 0.0; }
            dev::pcr_row(a0, c0, d0, la0, lc0, ld0, ua0, uc0, ud0, bad);
            dev::pcr_row(a1, c1, d1, la1, lc1, ld1, ua1, uc1, ud1, bad);
        }
    }
    if (valid) {
        X[(size_t)(2 * p) * nb + kl] = d0;
        X[(size_t)(2 * p + 1) * nb + kl] = d1;
        if (bad) atomicOr(err, 1);
    }
}

// Stage B, sequential variant: one lane per system eliminates its 2P
// unit-diagonal interface rows top-down and substitutes bottom-up (any P).
__global__ void __launch_bounds__(256)
k_stage_b_seq(const double *red, double *X, double *scratch, int64_t nb, int P, int *err) {
    const int64_t kl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kl >= nb) return;
    const int R2 = 2 * P;
    bool bad = false;
    // forward: row i -> x_i + g_i x_{i+1} = e_i (g, e kept in scratch, row-major by system)
    double gp = 0.0, ep = 0.0;
    for (int i = 0; i < R2; ++i) {
        const int p = i >> 1, v = (i & 1) * 3;
        const double a = red[red_at(v, p, kl, P, nb)], c = red[red_at(v + 1, p, kl, P, nb)];
        const double dd = red[red_at(v + 2, p, kl, P, nb)];
        const double piv = 1.0 - (i > 0 ? a * gp : 0.0);
        bad |= dev::bad_pivot(piv);
        const double ib = 1.0 / piv;
        gp = c * ib;
        ep = (dd - (i > 0 ? a * ep : 0.0)) * ib;
        scratch[(size_t)i * nb + kl] = gp;
        X[(size_t)i * nb + kl] = ep;
    }
    double xn = X[(size_t)(R2 - 1) * nb + kl];
    for (int i = R2 - 2; i >= 0; --i) {
        xn = X[(size_t)i * nb + kl] - scratch[(size_t)i * nb + kl] * xn;
        X[(size_t)i * nb + kl] = xn;
    }
    if (bad) atomicOr(err, 1);
}

template <typename T, bool SHARED_FACTORS>
__global__ void __launch_bounds__(256)
k_stage_c(SysMap map, T *__restrict__ x, const T *__restrict__ ws_d, const T *__restrict__ ws_a,
          const T *__restrict__ ws_c, const double *__restrict__ X, int64_t k_begin, int64_t nb,
          int P) {
    const int64_t kl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (kl >= nb) return;
    const dev::LaneSys sys = dev::lane_system(map, k_begin + kl);
    const PartRange pr = part_range(map.n, P, p);
    const int64_t rs = map.row_stride;
    const T xf = (T)X[(size_t)(2 * p) * nb + kl];
    T xn = (T)X[(size_t)(2 * p + 1) * nb + kl];
    const int64_t fk = SHARED_FACTORS ? 0 : kl;
    const int64_t fstride = SHARED_FACTORS ? 1 : nb;
    x[sys.base + (pr.start + pr.m - 1) * rs] = xn;
#pragma unroll 4
    for (int j = pr.m - 2; j >= 1; --j) {
        const int64_t r = pr.start + j;
        xn = ws_d[r * nb + kl] - ws_a[r * fstride + fk] * xf - ws_c[r * fstride + fk] * xn;
        x[sys.base + r * rs] = xn;
    }
    x[sys.base + pr.start * rs] = xf;
}

template <typename T>
hipError_t launch_a_t(const SysMap &map, const Coef &coef, const void *d, void *ws_d, void *ws_a,
                      void *ws_c, double *red, int64_t k_begin, int64_t nb, int P, bool shared_f,
                      int *err, hipStream_t st) {
    const dim3 grid((unsigned)((nb + 255) / 256), (unsigned)P);
    const bool like_d = coef.mode == TDMA_COEF_LIKE_D, shift = coef.shift != nullptr;
#define TDMA_A(LD, SH, SF)                                                                      \
    if (like_d == LD && shift == SH && shared_f == SF) {                                        \
        hipLaunchKernelGGL((k_stage_a<T, LD, SH, SF>), grid, dim3(256), 0, st, map, coef,       \
                           (const T *)d, (T *)ws_d, (T *)ws_a, (T *)ws_c, red, k_begin, nb, P, err); \
        return hipGetLastError();                                                               \
    }
    TDMA_A(true, false, false)
    TDMA_A(true, true, false)
    TDMA_A(false, false, false)
    TDMA_A(false, true, false)
    TDMA_A(false, false, true)
#undef TDMA_A
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_stage_a(int dtype, const SysMap &map, const Coef &coef, const void *d,
                          void *ws_d, void *ws_a, void *ws_c, double *red, int64_t k_begin,
                          int64_t nb, int P, bool shared_factors, int *err, hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    if (dtype == TDMA_F64)
        return launch_a_t<double>(map, coef, d, ws_d, ws_a, ws_c, red, k_begin, nb, P,
                                  shared_factors, err, st);
    return launch_a_t<float>(map, coef, d, ws_d, ws_a, ws_c, red, k_begin, nb, P, shared_factors,
                             err, st);
}

hipError_t launch_stage_b(const double *red, double *X, double *scratch, int64_t nb, int P,
                          int *err, hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    if (P <= 64 && (P & (P - 1)) == 0) {
        int P_log2 = 0;
        while ((1 << P_log2) < P) ++P_log2;
        const int64_t lanes = nb * P;
        hipLaunchKernelGGL(k_stage_b_pcr, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st,
                           red, X, nb, P, P_log2, err);
    } else {
        hipLaunchKernelGGL(k_stage_b_seq, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, red,
                           X, scratch, nb, P, err);
    }
    return hipGetLastError();
}

hipError_t launch_stage_c(int dtype, const SysMap &map, void *x, const void *ws_d,
                          const void *ws_a, const void *ws_c, const double *X, int64_t k_begin,
                          int64_t nb, int P, bool shared_factors, hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nb + 255) / 256), (unsigned)P);
#define TDMA_C(T, SF)                                                                          \
    hipLaunchKernelGGL((k_stage_c<T, SF>), grid, dim3(256), 0, st, map, (T *)x, (const T *)ws_d, \
                       (const T *)ws_a, (const T *)ws_c, X, k_begin, nb, P)
    if (dtype == TDMA_F64) {
        if (shared_factors) TDMA_C(double, true); else TDMA_C(double, false);
    } else {
        if (shared_factors) TDMA_C(float, true); else TDMA_C(float, false);
    }
#undef TDMA_C
    return hipGetLastError();
}

}  // namespace tdma
