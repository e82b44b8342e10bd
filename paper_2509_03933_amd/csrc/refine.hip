// Precision form: FP32 sweeps with FP64 iterative refinement, fused per tile.
//
// Per tile, on chip: the FP64 right-hand side d and solution x stay in
// registers; the partition factors (pivot reciprocals g, h = a g, the
// back-substitution factors a^, c^) are built once in FP32; then
//     x = 0;  r = d;  repeat 1 + iters times:
//         solve A e = r with the FP32 factors (Stage A/C in FP32, the 2P-row
//         interface solve in FP64), x += e, r = d - A x  (FP64).
// The residual needs each partition's outer neighbours, exchanged through
// LDS.  After the last step a system is converged if max|e| <= tol max|x|;
// systems that are not are appended to a device list that the FP64 fused
// kernel re-solves (the fallback), and the tile reports its largest
// relative correction.
#include "refine.h"
#include "tile.hip.h"

namespace tdma {
namespace {

using dev::Iface;
using dev::LaneSys;

template <int M, bool LIKE_D, bool SHIFT, bool CONTIG>
__global__ void __launch_bounds__(512)
k_refine(SysMap map, Coef coef, const double *d, double *x, int S_log2, int P, int iters,
         double tol, RefineState *state) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int S = 1 << S_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t n = map.n;
    const int64_t k0 = dev::xcd_tile(blockIdx.x, gridDim.x) << S_log2;
    const LaneSys sys = dev::lane_system(map, k0 + s);
    const int rows_here = (int)(sys.nrows - r0 < 0 ? 0 : (sys.nrows - r0 > M ? M : sys.nrows - r0));
    const double *A = (const double *)coef.a, *B = (const double *)coef.b,
                 *C = (const double *)coef.c;
    // LDS: [0, region0) PCR scratch or staging; XB = S x (2P+1) doubles; the
    // shared coefficient tables (3 x P*M doubles, shared mode); the tile table
    const int R = P * M;
    const size_t pcr_b = dev::pcr_lds_bytes(S, P);
    const size_t stg_b = CONTIG ? (((size_t)S * (R + 1) * 8 + 15) & ~(size_t)15) : 0;
    const size_t region0 = pcr_b > stg_b ? pcr_b : stg_b;
    double *XB = reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + region0);
    const int xpitch = 2 * P + 1;
    double *CT = reinterpret_cast<double *>(reinterpret_cast<char *>(XB) +
                                            (((size_t)S * xpitch * 8 + 15) & ~(size_t)15));
    const size_t ct_b = LIKE_D ? 0 : (size_t)3 * R * 8;
    dev::TileSysLds *tsys = reinterpret_cast<dev::TileSysLds *>(reinterpret_cast<char *>(CT) + ct_b);
    // Loads in the order their consumers need them: the shift and the shared
    // operator's rows (the FP32 factors need only these), then the tile's
    // right-hand sides (and per-row coefficients), which stay in flight while
    // the shared rows go to LDS.
    double shv = 0.0;
    if constexpr (SHIFT) {
        shv = ((const double *)coef.shift)[sys.valid ? sys.id : 0];
        if (!sys.valid) shv = 0.0;
    }
    dev::RowRegs<1> rr;
    if constexpr (!LIKE_D) dev::rows_prefetch<double, 1>(coef, n, rr);
    __builtin_amdgcn_sched_barrier(0);

    double dv[M], av[LIKE_D ? M : 1], bv[LIKE_D ? M : 1], cv[LIKE_D ? M : 1];
    double *stg = lds;
    const float invR = 1.0f / (float)R;
    if constexpr (!CONTIG) {
        // branch-free: the row index stops at the system's last row, padding
        // rows are replaced after the loads
        const int64_t rs = map.row_stride;
        const int64_t last = sys.nrows > 0 ? sys.nrows - 1 : 0;
        const int64_t first = r0 < last ? r0 : last;
        const int adv = (int)(last - first < M ? last - first : M);
        int64_t idx = (sys.valid ? sys.base : 0) + first * rs;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            dv[j] = d[idx];
            if constexpr (LIKE_D) {
                av[j] = A[idx]; bv[j] = B[idx]; cv[j] = C[idx];
            }
            idx += j < adv ? rs : 0;
        }
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j >= rows_here) {
                dv[j] = 0.0;
                if constexpr (LIKE_D) { av[j] = 0.0; bv[j] = 1.0; cv[j] = 0.0; }
            }
    } else {
        if (tid < S) {
            const LaneSys q = dev::lane_system(map, k0 + tid);
            tsys[tid].base = q.base;
            tsys[tid].nrows = q.nrows;
        }
        __syncthreads();
        dev::stage_load<double, M>(tsys, d, S, R, invR, dv);
        if constexpr (LIKE_D) {
            dev::stage_load<double, M>(tsys, A, S, R, invR, av);
            dev::stage_load<double, M>(tsys, B, S, R, invR, bv);
            dev::stage_load<double, M>(tsys, C, S, R, invR, cv);
        }
    }
    // one copy of the shared FP64 operator per workgroup, corners removed,
    // identity rows past n
    if constexpr (!LIKE_D) dev::rows_commit<double, 1>(CT, coef, n, R, rr);
    if constexpr (CONTIG) {
        double ld[M];
#pragma unroll
        for (int j = 0; j < M; ++j) ld[j] = dv[j];
        dev::stage_put<double, M>(stg, tsys, 0.0, S, R, R + 1, invR, s, r0, ld, dv);
        if constexpr (LIKE_D) {
#pragma unroll
            for (int j = 0; j < M; ++j) ld[j] = av[j];
            dev::stage_put<double, M>(stg, tsys, 0.0, S, R, R + 1, invR, s, r0, ld, av);
#pragma unroll
            for (int j = 0; j < M; ++j) ld[j] = bv[j];
            dev::stage_put<double, M>(stg, tsys, 1.0, S, R, R + 1, invR, s, r0, ld, bv);
#pragma unroll
            for (int j = 0; j < M; ++j) ld[j] = cv[j];
            dev::stage_put<double, M>(stg, tsys, 0.0, S, R, R + 1, invR, s, r0, ld, cv);
        }
    }
    // FP64 coefficients of local row j (identity beyond the system)
    auto coefs = [&](int j, double &a, double &b, double &c) {
        const int64_t r = r0 + j;
        if constexpr (LIKE_D) {
            if (j < rows_here) {
                a = r == 0 ? 0.0 : av[j];
                b = bv[j];
                c = r == n - 1 ? 0.0 : cv[j];
                if constexpr (SHIFT) b += shv;
            } else {
                a = 0.0; b = 1.0; c = 0.0;
            }
        } else {
            a = CT[r]; b = CT[R + r]; c = CT[2 * R + r];
            if constexpr (SHIFT) {
                if (j < rows_here) b += shv;
            }
        }
    };

    // FP32 factors
    float g[M], fa[M], fc[M];
    bool bad = false;
    float piv;
    {
        double a, b, c;
        coefs(0, a, b, c);
        piv = (float)b;
        bad |= dev::bad_pivot(piv);
        g[0] = dev::recip(piv);
        fa[0] = (float)a * g[0]; fc[0] = (float)c * g[0];
        coefs(1, a, b, c);
        piv = (float)b;
        bad |= dev::bad_pivot(piv);
        g[1] = dev::recip(piv);
        fa[1] = (float)a * g[1]; fc[1] = (float)c * g[1];
#pragma unroll
        for (int j = 2; j < M; ++j) {
            coefs(j, a, b, c);
            piv = (float)b - (float)a * fc[j - 1];
            bad |= dev::bad_pivot(piv);
            g[j] = dev::recip(piv);
            fa[j] = -((float)a * g[j]) * fa[j - 1];
            fc[j] = (float)c * g[j];
        }
    }
    float pi = 1.0f, at1 = 0.0f;
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        at1 += pi * fa[j];
        pi = -fc[j] * pi;
    }
    const float ct1 = -pi;
    const double den = 1.0 - (double)fc[0] * (double)at1;
    bad |= dev::bad_pivot(den);
    const double rho = 1.0 / den;
    Iface f;
    f.fa = rho * (double)fa[0];
    f.fc = -rho * (double)fc[0] * (double)ct1;
    f.la = (double)fa[M - 1];
    f.lc = (double)fc[M - 1];
    const double K0 = rho * (double)g[0], K1 = rho * (double)fc[0];
    const bool wave_pcr = P <= 64 && (P & (P - 1)) == 0;
    const int P_log2 = __builtin_ctz(P);

    double xv[M];
    float e[M];
    float ecur = 0.0f, eprev = 0.0f;   // largest entry of the last two corrections
#pragma unroll
    for (int j = 0; j < M; ++j) xv[j] = 0.0;
    for (int it = 0; it <= iters; ++it) {
        // r = d - A x (FP64); first pass r = d
        if (it == 0) {
#pragma unroll
            for (int j = 0; j < M; ++j) e[j] = (float)dv[j];
        } else {
            __syncthreads();
            XB[s * xpitch + 2 * p] = xv[0];
            XB[s * xpitch + 2 * p + 1] = xv[M - 1];
            __syncthreads();
            const double xlo = p > 0 ? XB[s * xpitch + 2 * p - 1] : 0.0;
            const double xhi = p < P - 1 ? XB[s * xpitch + 2 * p + 2] : 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                double a, b, c;
                coefs(j, a, b, c);
                const double xm = j == 0 ? xlo : xv[j > 0 ? j - 1 : 0];
                const double xp = j == M - 1 ? xhi : xv[j < M - 1 ? j + 1 : M - 1];
                e[j] = (float)(dv[j] - a * xm - b * xv[j] - c * xp);
            }
        }
        // solve A e = r with the FP32 factors
        const float r0v = e[0];
        e[1] = g[1] * e[1];
#pragma unroll
        for (int j = 2; j < M; ++j) {
            double a, b, c;
            coefs(j, a, b, c);
            e[j] = (e[j] - (float)a * e[j - 1]) * g[j];
        }
        float dt1 = 0.0f;
        pi = 1.0f;
#pragma unroll
        for (int j = 1; j <= M - 2; ++j) {
            dt1 += pi * e[j];
            pi = -fc[j] * pi;
        }
        f.fd = K0 * (double)r0v - K1 * (double)dt1;
        f.ld = (double)e[M - 1];
        double xf, xl;
        if (wave_pcr)
            dev::pcr_interface_wave(lds, S, s, p, P, P_log2, f, xf, xl, bad);
        else
            dev::pcr_interface(lds, S, s, p, P, f, xf, xl, bad);
        e[M - 1] = (float)xl;
#pragma unroll
        for (int j = M - 2; j >= 1; --j) e[j] = e[j] - fa[j] * (float)xf - fc[j] * e[j + 1];
        e[0] = (float)xf;
        eprev = ecur;
        ecur = 0.0f;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            xv[j] += (double)e[j];
            ecur = fmaxf(ecur, fabsf(e[j]));
        }
    }
    // convergence per system (refine_ratio) from the largest entries of the
    // last two corrections and of x over the system's partitions
    double xmax = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) xmax = fmax(xmax, fabs(xv[j]));
    // a zero or non-finite FP32 pivot sends the system to the FP64 fallback
    if (bad) ecur = __builtin_huge_valf();
    __syncthreads();
    XB[s * xpitch + 2 * p] = pack_e(ecur, eprev);
    XB[s * xpitch + 2 * p + 1] = xmax;
    __syncthreads();
    // the partition-0 lanes (threads 0 .. S-1) judge their systems; their
    // wavefronts then record misses with one atomicAdd and the largest ratio
    // with at most one atomicMax each
    if ((tid & ~63) < S) {
        double rel = 0.0;
        bool miss = false;
        if (p == 0 && sys.valid) {
            float em = 0.0f, ep = 0.0f;
            double xm = 0.0;
            for (int q = 0; q < P; ++q) {
                float eq, epq;
                unpack_e(XB[s * xpitch + 2 * q], eq, epq);
                em = fmaxf(em, eq);
                ep = fmaxf(ep, epq);
                xm = fmax(xm, XB[s * xpitch + 2 * q + 1]);
            }
            rel = refine_ratio(state->criterion, iters, (double)em, (double)ep, xm);
            miss = !(rel <= tol);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            if (off < (int)blockDim.x) rel = fmax(rel, __shfl_xor(rel, off));
        const unsigned long long ball = __ballot(miss);
        if ((tid & 63) == 0) fold_max_rel(state, rel);
        if (ball) {
            unsigned long long first = 0;
            if ((tid & 63) == 0) first = atomicAdd(&state->not_converged, (unsigned long long)__popcll(ball));
            first = __shfl(first, 0);
            if (miss) {
                const unsigned long long slot = first + __popcll(ball & __lanemask_lt());
                if (state->fallback_list && slot < (unsigned long long)state->list_capacity)
                    state->fallback_list[slot] = (int32_t)sys.id;
            }
        }
    }
    if constexpr (!CONTIG) {
        double *px = x + sys.base + (int64_t)r0 * map.row_stride;
        const int64_t rs = map.row_stride;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < rows_here) px[j * rs] = xv[j];
    } else {
        dev::stage_out<double, M>(lds, tsys, x, S, R, R + 1, 1.0f / (float)R, s, r0, xv);
    }
}

// Residual r = d - a x_{-} - b x - c x_{+} accumulated in double-double
// (error-free product via FMA, error-free sums) and rounded once, so the
// residual of an ill-conditioned system is accurate to the last bit even when
// its terms cancel.  Contraction is off inside: the error-free transforms
// rely on every add being rounded on its own.
__device__ __forceinline__ double residual_dd(double d, double a, double xm, double b, double x0,
                                              double c, double xp) {
#pragma clang fp contract(off)
    double hi = d, lo = 0.0;
    auto acc = [&](double u, double v) {
        const double pr = -u * v;
        const double pe = __builtin_fma(-u, v, -pr);   // exact: -u*v = pr + pe
        const double s = hi + pr;
        const double bb = s - hi;
        const double t = (hi - (s - bb)) + (pr - bb);  // exact: hi + pr = s + t
        hi = s;
        lo = lo + (t + pe);
    };
    acc(a, xm);
    acc(b, x0);
    acc(c, xp);
    return hi + lo;
}

// Polishing of listed systems (the FP64 fallback): `steps` rounds of
// double-double residual and FP64 on-chip correction solve, one system per
// block of P lanes (M rows each).  Grid-stride over the device-side count.
template <int M, bool LIKE_D, bool SHIFT>
__global__ void __launch_bounds__(512)
k_polish(SysMap map, Coef coef, const double *d, double *x, const int32_t *list,
         const unsigned long long *count, int64_t capacity, int P, int steps) {
    extern __shared__ double lds[];
    const int p = threadIdx.x;
    const int r0 = p * M;
    const int64_t n = map.n;
    const int64_t cnt = (int64_t)*count < capacity ? (int64_t)*count : capacity;
    const double *A = (const double *)coef.a, *B = (const double *)coef.b,
                 *C = (const double *)coef.c;
    double *XB = lds + 3 * (2 * P + 1);          // after the PCR scratch (S = 1)
    const bool wave_pcr = P <= 64 && (P & (P - 1)) == 0;
    for (int64_t k = blockIdx.x; k < cnt; k += gridDim.x) {
        const int64_t id = list[k];
        const int64_t s1 = id / map.nsys0, s0 = id - s1 * map.nsys0;
        const int64_t sbase = s0 * map.sys_stride0 + s1 * map.sys_stride1;
        const int64_t rs = map.row_stride;
        const double shv = SHIFT ? ((const double *)coef.shift)[id] : 0.0;
        double av[M], bv[M], cv[M], dv[M], xv[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int64_t r = r0 + j;
            if (r < n) {
                const int64_t idx = sbase + r * rs;
                dv[j] = d[idx];
                xv[j] = x[idx];
                av[j] = r == 0 ? 0.0 : (LIKE_D ? A[idx] : A[r]);
                bv[j] = (LIKE_D ? B[idx] : B[r]) + shv;
                cv[j] = r == n - 1 ? 0.0 : (LIKE_D ? C[idx] : C[r]);
            } else {
                dv[j] = 0.0; xv[j] = 0.0; av[j] = 0.0; bv[j] = 1.0; cv[j] = 0.0;
            }
        }
        bool bad = false;
        for (int step = 0; step < steps; ++step) {
            __syncthreads();
            XB[2 * p] = xv[0];
            XB[2 * p + 1] = xv[M - 1];
            __syncthreads();
            const double xlo = p > 0 ? XB[2 * p - 1] : 0.0;
            const double xhi = p < P - 1 ? XB[2 * p + 2] : 0.0;
            double rv[M], wa[M], wc[M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double xm = j == 0 ? xlo : xv[j > 0 ? j - 1 : 0];
                const double xp = j == M - 1 ? xhi : xv[j < M - 1 ? j + 1 : M - 1];
                rv[j] = residual_dd(dv[j], av[j], xm, bv[j], xv[j], cv[j], xp);
                wa[j] = av[j];
                wc[j] = cv[j];
            }
            const dev::Iface f = dev::reduce_partition<double, M>(wa, bv, wc, rv, bad);
            double xf, xl;
            if (wave_pcr)
                dev::pcr_interface_wave(lds, 1, 0, p, P, __builtin_ctz(P), f, xf, xl, bad);
            else
                dev::pcr_interface(lds, 1, 0, p, P, f, xf, xl, bad);
            dev::substitute_partition<double, M>(wa, wc, rv, xf, xl);
#pragma unroll
            for (int j = 0; j < M; ++j) xv[j] += rv[j];
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int64_t r = r0 + j;
            if (r < n) x[sbase + r * rs] = xv[j];
        }
    }
}

__global__ void k_refine_init(RefineState *state, int32_t *list, int64_t capacity, int criterion,
                              int *err) {
    if (err) *err = 0;
    state->not_converged = 0ull;
    state->max_rel_bits = 0ull;
    state->fallback_list = list;
    state->list_capacity = capacity;
    state->criterion = criterion;
}

template <int M>
hipError_t launch_m(const SysMap &map, const Coef &coef, const TileShape &sh, const double *d,
                    double *x, int iters, double tol, RefineState *state, size_t lds, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    const bool like_d = coef.mode == TDMA_COEF_LIKE_D, shift = coef.shift != nullptr;
#define TDMA_R(LD, SH, CT)                                                                       \
    if (like_d == LD && shift == SH && sh.contig == CT) {                                        \
        hipLaunchKernelGGL((k_refine<M, LD, SH, CT>), dim3((unsigned)blocks), dim3(sh.threads()), \
                           lds, st, map, coef, d, x, sh.S_log2, sh.P, iters, tol, state);        \
        return hipGetLastError();                                                                \
    }
    if constexpr (M == 8) {   // per-row coefficients only with M = 8
        TDMA_R(true, false, false)
        TDMA_R(true, true, false)
        TDMA_R(true, false, true)
        TDMA_R(true, true, true)
    }
    TDMA_R(false, false, false)
    TDMA_R(false, true, false)
    TDMA_R(false, false, true)
    TDMA_R(false, true, true)
#undef TDMA_R
    return hipErrorInvalidValue;
}

}  // namespace

size_t refine_lds_bytes(const TileShape &sh, bool like_d) {
    const int S = 1 << sh.S_log2;
    const size_t pcr_b = dev::pcr_lds_bytes(S, sh.P);
    const size_t stg_b = sh.contig ? (((size_t)S * (sh.P * sh.M + 1) * 8 + 15) & ~(size_t)15) : 0;
    const size_t region0 = pcr_b > stg_b ? pcr_b : stg_b;
    const size_t ct_b = like_d ? 0 : (size_t)3 * sh.P * sh.M * 8;
    return region0 + (((size_t)S * (2 * sh.P + 1) * 8 + 15) & ~(size_t)15) + ct_b + 16 * (size_t)S;
}

int refine_max_threads(int) { return 512; }

bool refine_supported(const TileShape &sh, bool like_d) {
    if (sh.M != 8 && sh.M != 16) return false;
    if (like_d && sh.M != 8) return false;
    if (sh.P < 1 || sh.threads() > refine_max_threads(sh.M)) return false;
    return refine_lds_bytes(sh, like_d) <= 160 * 1024;
}

hipError_t launch_refine_init(RefineState *state, int32_t *list, int64_t capacity, int criterion,
                              int *clear_err, hipStream_t st) {
    hipLaunchKernelGGL(k_refine_init, dim3(1), dim3(1), 0, st, state, list, capacity, criterion,
                       clear_err);
    return hipGetLastError();
}

hipError_t launch_refine(const SysMap &map, const Coef &coef, const TileShape &sh, const double *d,
                         double *x, int iters, double tol, RefineState *state, hipStream_t st) {
    const size_t lds = refine_lds_bytes(sh, coef.mode == TDMA_COEF_LIKE_D);
    if (sh.M == 8) return launch_m<8>(map, coef, sh, d, x, iters, tol, state, lds, st);
    if (sh.M == 16) return launch_m<16>(map, coef, sh, d, x, iters, tol, state, lds, st);
    return hipErrorInvalidValue;
}

int polish_partitions(int64_t n) {
    int P = 1;
    while ((int64_t)P * 8 < n) P <<= 1;
    return P;
}

hipError_t launch_polish(const SysMap &map, const Coef &coef, const double *d, double *x,
                         const int32_t *list, const unsigned long long *count, int64_t capacity,
                         int steps, hipStream_t st) {
    const int P = polish_partitions(map.n);
    if (P > 512) return hipErrorInvalidValue;
    const size_t lds = dev::pcr_lds_bytes(1, P) + (size_t)(2 * P + 2) * sizeof(double);
    const unsigned grid = (unsigned)(capacity < 2048 ? capacity : 2048);
    if (grid == 0) return hipSuccess;
    const bool like_d = coef.mode == TDMA_COEF_LIKE_D, shift = coef.shift != nullptr;
#define TDMA_PO(LD, SH)                                                                     \
    if (like_d == LD && shift == SH) {                                                      \
        hipLaunchKernelGGL((k_polish<8, LD, SH>), dim3(grid), dim3(P), lds, st, map, coef, d, x, \
                           list, count, capacity, P, steps);                                \
        return hipGetLastError();                                                           \
    }
    TDMA_PO(true, false)
    TDMA_PO(true, true)
    TDMA_PO(false, false)
    TDMA_PO(false, true)
#undef TDMA_PO
    return hipErrorInvalidValue;
}

}  // namespace tdma
