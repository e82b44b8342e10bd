// Shared-operator fused solve (the ADI and Poisson-line case where every
// system of a launch has the same a, b, c; the coefficient matrix depends only
// on the grid spacing).  The Stage A/B/C arithmetic is that of tile.hip.h, but
// everything that depends only on the coefficients is computed once per
// workgroup into LDS tables while the tile's right-hand sides are in flight:
//   per partition row j:  G_j, H_j   (d^_j = G_j d_j - H_j d^_{j-1}),
//                         pi_j       (running products of the row-1 spike),
//                         a^_j, c^_j (back-substitution factors),
//   per partition:        K0, K1     (first interface RHS = K0 d_0 - K1 dt1)
//                         and the four interface coefficients,
//   per PCR step and interface row: the pre-step couplings and 1/beta.
// The per-system work is then about five FP64 operations per row, and the
// interface solve exchanges one value per row instead of three.
// Kernels: k_shared (one tile per workgroup), k_shared_stream (strided
// layouts: resident workgroups walk the tiles), k_shared_cstream (the same
// for contiguous rows of consecutive systems, through an LDS transpose),
// k_shared_refine (the precision form), k_copy_stream (the streaming
// kernel's memory traffic alone, for measurement).
#include <type_traits>

#include "refine.h"
#include "tile.hip.h"
#include "walk.hip.h"

namespace tdma {
namespace {

using dev::Ident;
using dev::LaneSys;
using dev::TileSysLds;

// LDS carve-up, byte offsets (each region 16-byte aligned):
//   gh, ac : P x (M+1) pairs of T, {g_j, h_j} and {a^_j, c^_j}: one LDS read
//            per row for each pair; the partition pitch of M+1 pairs puts the
//            two partitions a wavefront reads on different banks
//   pi     : P x (M+1) values of T
//   part   : 6 x P doubles (K0, K1, AF, GF, AL, GL)
//   qa     : 3 x nsteps x 2P doubles (pre-step a, c and 1/beta)
//   xd     : S x (2P+2) doubles (interface right-hand sides, read and written
//            as pairs; the even pitch keeps both lane mappings conflict-free)
//   co     : 3 x P*M doubles (the tile's a, b, c rows, corners removed)
//   end    : staging of the contiguous-row variant starts here
struct SharedLds {
    size_t gh, ac, pi, part, qa, xd, co, end;
    int nsteps;
};

template <typename T> struct PairOf;
template <> struct PairOf<double> { using type = double2; };
template <> struct PairOf<float> { using type = float2; };

__host__ __device__ inline int ilog2i(int v) {
    int r = 0;
    while ((1 << (r + 1)) <= v) ++r;
    return r;
}

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

__host__ __device__ inline int xd_pitch(int P) { return 2 * P + 2; }

// co_transient: the coefficient rows are read only while the tables are
// built (k_shared, k_shared_stream), so they share the space of the
// interface exchange, which is first written after that build's barrier;
// the precision form reads them for every residual and keeps them apart.
__host__ __device__ inline SharedLds shared_layout(size_t esz, int M, int P, int S,
                                                   bool co_transient = true) {
    SharedLds L;
    const size_t pairs = align16((size_t)P * (M + 1) * 2 * esz);
    L.gh = 0;
    L.ac = L.gh + pairs;
    L.pi = L.ac + pairs;
    L.part = align16(L.pi + (size_t)P * (M + 1) * esz);
    L.nsteps = ilog2i(2 * P);
    if ((1 << L.nsteps) < 2 * P) ++L.nsteps;
    L.qa = align16(L.part + 6 * (size_t)P * 8);
    L.xd = align16(L.qa + 3 * (size_t)L.nsteps * 2 * P * 8);
    const size_t xd_bytes = (size_t)S * xd_pitch(P) * 8, co_bytes = 3 * (size_t)P * M * 8;
    if (co_transient) {
        L.co = L.xd;
        L.end = align16(L.xd + (xd_bytes > co_bytes ? xd_bytes : co_bytes));
    } else {
        L.co = align16(L.xd + xd_bytes);
        L.end = align16(L.co + co_bytes);
    }
    return L;
}

// Read side of one partition's factor tables.
template <typename T>
struct PartTab {
    const typename PairOf<T>::type *gh, *ac;
    const T *pi;
    __device__ PartTab(const SharedLds &L, const char *base, int p, int M) {
        using P2 = typename PairOf<T>::type;
        gh = reinterpret_cast<const P2 *>(base + L.gh) + p * (M + 1);
        ac = reinterpret_cast<const P2 *>(base + L.ac) + p * (M + 1);
        pi = reinterpret_cast<const T *>(base + L.pi) + p * (M + 1);
    }
};

// contiguous-row variant: staging of S x (P*M+1) values of T, then S tile entries
__host__ __device__ inline size_t shared_stage_off(const SharedLds &L) { return L.end; }
__host__ __device__ inline size_t shared_tsys_off(const SharedLds &L, size_t esz, int M, int P, int S) {
    return align16(L.end + (size_t)S * ((size_t)P * M + 1) * esz);
}

template <typename T, int M>
constexpr int shared_max_threads() { return (int)sizeof(T) * M >= 192 ? 512 : 1024; }

// Coefficient rows held in registers per thread (tile rows P*M over S*P
// threads: M/S rows each; rows beyond CR per thread are loaded late).
template <int M>
constexpr int shared_cr() { return M >= 32 ? 2 : 1; }

// Right-hand sides of a lane's M rows in a strided layout, loaded without
// branches so that the loads form one straight run behind the coefficient
// loads (the load counter then stays exact): the pointer stops advancing at
// the system's last row and a lane past the last system reads the start of
// the array.  Rows past the system's end hold garbage until mask_rows zeroes
// them, which the kernels do only when the rows are consumed, so nothing
// waits on these loads early.  OffT is the type of the byte offsets from the
// array's start: uint32_t when the whole array spans less than 4 GiB (one
// register per address, the base stays scalar), else int64_t.  Every element
// is read once per solve, so the loads (and store_rows' stores) carry the
// non-temporal hint: measured on the 256^3 ADI sweep, 59.0 -> 56.0 us for
// the solve and 54.6 -> 51.2 us for the same pattern with no arithmetic.
template <typename T, int M, typename OffT>
__device__ __forceinline__ void load_rows(const T *d, const LaneSys &sys, int64_t rs, int r0,
                                          T (&dv)[M]) {
    const int64_t last = sys.nrows > 0 ? sys.nrows - 1 : 0;
    const int64_t first = r0 < last ? r0 : last;
    const int adv = (int)(last - first < M ? last - first : M);   // rows the pointer may advance
    const char *b = reinterpret_cast<const char *>(d);
    const OffT step = (OffT)(rs * (int64_t)sizeof(T));
    OffT off = (OffT)(((sys.valid ? sys.base : 0) + first * rs) * (int64_t)sizeof(T));
#pragma unroll
    for (int j = 0; j < M; ++j) {
        dv[j] = __builtin_nontemporal_load(reinterpret_cast<const T *>(b + off));
        off += j < adv ? step : OffT(0);
    }
}

// Rows of the lane's partition that lie inside its system (0..M).
__device__ __forceinline__ int rows_in(const LaneSys &sys, int r0, int M) {
    return (int)(sys.nrows - r0 < 0 ? 0 : (sys.nrows - r0 > M ? M : sys.nrows - r0));
}

template <typename T, int M>
__device__ __forceinline__ void mask_rows(int rows_here, T (&dv)[M]) {
#pragma unroll
    for (int j = 0; j < M; ++j)
        if (j >= rows_here) dv[j] = T(0);
}

// Steps shared by the shared-operator kernels: copy the tile's coefficient
// rows into LDS, build the per-partition factor tables (one lane per
// partition, FP64 arithmetic, stored as T; the coefficient arrays hold CT),
// and record the coefficient history of the interface PCR (first wavefront).
// Every thread calls it.
template <typename T, typename CT, int M>
__device__ __forceinline__ void shared_tables(const Coef &coef, int64_t n, const SharedLds &L,
                                              char *base, int tid, int s, int p, int P,
                                              const dev::RowRegs<shared_cr<M>()> &cr, bool &bad) {
    using P2 = typename PairOf<T>::type;
    const int r0 = p * M;
    const int pitch = M + 1;
    P2 *GH = reinterpret_cast<P2 *>(base + L.gh);
    P2 *AC = reinterpret_cast<P2 *>(base + L.ac);
    T *PI = reinterpret_cast<T *>(base + L.pi);
    double *PT = reinterpret_cast<double *>(base + L.part);
    double *K0 = PT, *K1 = PT + P, *AF = PT + 2 * P, *GF = PT + 3 * P, *AL = PT + 4 * P,
           *GL = PT + 5 * P;
    double *QA = reinterpret_cast<double *>(base + L.qa);
    double *QC = QA + L.nsteps * 2 * P, *QB = QC + L.nsteps * 2 * P;
    // coefficient tables, one lane per partition (FP64 arithmetic), from a
    //    copy of the tile's coefficient rows in LDS (corners and padding removed)
    dev::rows_commit<CT, shared_cr<M>()>(reinterpret_cast<double *>(base + L.co), coef, n, P * M,
                                         cr);
    if (s == 0) {
        const double *CO = reinterpret_cast<const double *>(base + L.co);
        const int R = P * M;
        auto row = [&](int j, double &aj, double &bj, double &cj) {
            const int r = r0 + j;
            aj = CO[r];
            bj = CO[R + r];
            cj = CO[2 * R + r];
        };
        double a0, b0, c0, aj, bj, cj;
        row(0, a0, b0, c0);
        bad |= dev::bad_pivot(b0);
        const double ib0 = dev::recip(b0);
        const double ah0 = a0 * ib0, ch0 = c0 * ib0;
        P2 *gh = GH + p * pitch, *ac = AC + p * pitch;
        T *pi_t = PI + p * pitch;
        gh[0] = P2{(T)ib0, T(0)}; pi_t[0] = T(0); ac[0] = P2{(T)ah0, (T)ch0};
        row(1, aj, bj, cj);
        bad |= dev::bad_pivot(bj);
        double gj = dev::recip(bj);
        double ahp = aj * gj, chp = cj * gj;
        gh[1] = P2{(T)gj, T(0)}; ac[1] = P2{(T)ahp, (T)chp};
        double pi = 1.0, at1 = 0.0;
        if (M > 2) { pi_t[1] = (T)pi; at1 += pi * ahp; pi = -chp * pi; }
#pragma unroll 1
        for (int j = 2; j < M; ++j) {
            row(j, aj, bj, cj);
            const double piv = bj - aj * chp;
            bad |= dev::bad_pivot(piv);
            gj = dev::recip(piv);
            const double hj = aj * gj;
            ahp = -hj * ahp;
            chp = cj * gj;
            gh[j] = P2{(T)gj, (T)hj}; ac[j] = P2{(T)ahp, (T)chp};
            if (j <= M - 2) { pi_t[j] = (T)pi; at1 += pi * ahp; pi = -chp * pi; }
        }
        pi_t[M - 1] = T(0);
        const double ct1 = -pi;
        const double den = 1.0 - ch0 * at1;
        bad |= dev::bad_pivot(den);
        const double rho = dev::recip(den);
        K0[p] = rho * ib0;
        K1[p] = rho * ch0;
        AF[p] = rho * ah0;
        GF[p] = -rho * ch0 * ct1;
        AL[p] = ahp;
        GL[p] = chp;
    }
    __syncthreads();
    // 3. coefficient history of the interface PCR (first wavefront; P <= 64)
    if (tid < 64) {
        const int lane = tid;
        const bool act = lane < P;
        double a0 = act ? AF[lane] : 0.0, c0 = act ? GF[lane] : 0.0;
        double a1 = act ? AL[lane] : 0.0, c1 = act ? GL[lane] : 0.0;
        int k = 0;
        for (int h = 1; h < 2 * P; h <<= 1, ++k) {
            double la0, lc0, la1, lc1, ua0, uc0, ua1, uc1;
            if (h == 1) {
                const bool has_lo = lane > 0 && act, has_hi = lane < P - 1 && act;
                const int lo = has_lo ? lane - 1 : lane, hi = has_hi ? lane + 1 : lane;
                const double m_a = __shfl(a1, lo), m_c = __shfl(c1, lo);
                const double p_a = __shfl(a0, hi), p_c = __shfl(c0, hi);
                la0 = has_lo ? m_a : 0.0; lc0 = has_lo ? m_c : 0.0;   // row 2l-1
                ua0 = a1; uc0 = c1;                                    // row 2l+1
                la1 = a0; lc1 = c0;                                    // row 2l
                ua1 = has_hi ? p_a : 0.0; uc1 = has_hi ? p_c : 0.0;   // row 2l+2
            } else {
                const int dl = h >> 1;
                const bool has_lo = lane >= dl && act, has_hi = lane + dl < P && act;
                const int lo = has_lo ? lane - dl : lane, hi = has_hi ? lane + dl : lane;
                const double x_a0 = __shfl(a0, lo), x_c0 = __shfl(c0, lo);
                const double x_a1 = __shfl(a1, lo), x_c1 = __shfl(c1, lo);
                const double y_a0 = __shfl(a0, hi), y_c0 = __shfl(c0, hi);
                const double y_a1 = __shfl(a1, hi), y_c1 = __shfl(c1, hi);
                la0 = has_lo ? x_a0 : 0.0; lc0 = has_lo ? x_c0 : 0.0;
                la1 = has_lo ? x_a1 : 0.0; lc1 = has_lo ? x_c1 : 0.0;
                ua0 = has_hi ? y_a0 : 0.0; uc0 = has_hi ? y_c0 : 0.0;
                ua1 = has_hi ? y_a1 : 0.0; uc1 = has_hi ? y_c1 : 0.0;
            }
            const double b0 = 1.0 - a0 * lc0 - c0 * ua0;
            const double b1 = 1.0 - a1 * lc1 - c1 * ua1;
            const double ib0 = dev::recip(b0), ib1 = dev::recip(b1);
            if (act) {
                bad |= dev::bad_pivot(b0) || dev::bad_pivot(b1);
                const int i0 = 2 * lane, i1 = i0 + 1, base_k = k * 2 * P;
                QA[base_k + i0] = a0; QC[base_k + i0] = c0; QB[base_k + i0] = ib0;
                QA[base_k + i1] = a1; QC[base_k + i1] = c1; QB[base_k + i1] = ib1;
            }
            const double na0 = -a0 * la0 * ib0, nc0 = -c0 * uc0 * ib0;
            const double na1 = -a1 * la1 * ib1, nc1 = -c1 * uc1 * ib1;
            a0 = na0; c0 = nc0; a1 = na1; c1 = nc1;
        }
    }
    __syncthreads();

}

// The value `v` of the lane DL below / above the caller's lane.  DPP: the
// lane DL positions lower / higher in the caller's row of 16 lanes (zero when
// that lane is outside the row), a VALU operand modifier instead of an LDS
// permute; valid when every system's interface lanes lie in one row.
// Otherwise a wavefront shuffle (the caller's own value when out of range).
template <int DL, bool DPP>
__device__ __forceinline__ double lane_below(double v, int lane) {
    if constexpr (DPP && DL < 16)
        return row_shift<DL, true>(v);
    else
        return __shfl(v, lane >= DL ? lane - DL : lane);
}

template <int DL, bool DPP>
__device__ __forceinline__ double lane_above(double v, int lane) {
    if constexpr (DPP && DL < 16)
        return row_shift<DL, false>(v);
    else
        return __shfl(v, lane + DL < 64 ? lane + DL : lane);
}

// The four neighbour values of one PCR step at distance DL: rows 2p and
// 2p+1 of the lanes DL below (x0, x1) and above (y0, y1).
template <int DL, bool DPP>
__device__ __forceinline__ void fetch4(double e0, double e1, int lane, double &x0, double &x1,
                                       double &y0, double &y1) {
    x0 = lane_below<DL, DPP>(e0, lane);
    x1 = lane_below<DL, DPP>(e1, lane);
    y0 = lane_above<DL, DPP>(e0, lane);
    y1 = lane_above<DL, DPP>(e1, lane);
}

// PCR over the right-hand sides e0 = row 2p, e1 = row 2p+1 of one system
// held by P consecutive lanes, with the recorded coefficient history (QA,
// QC: pre-step couplings, QB: 1/beta; rows 2p and 2p+1 are adjacent, read as
// pairs).  A loop, not unrolled, so each step's history is read in its step;
// the exchange distance picks its DPP form through a uniform switch.
template <bool DPP>
__device__ __forceinline__ void rhs_pcr(double &e0, double &e1, const double *QA, const double *QC,
                                        const double *QB, int P, int p2, int lane) {
#pragma unroll 1
    for (int k = 0; (1 << k) < 2 * P; ++k) {
        const int q = k * 2 * P + 2 * p2;
        const double2 qa = *reinterpret_cast<const double2 *>(QA + q);
        const double2 qc = *reinterpret_cast<const double2 *>(QC + q);
        const double2 qb = *reinterpret_cast<const double2 *>(QB + q);
        double l0, u0, l1, u1;
        if (k == 0) {
            const bool has_lo = p2 > 0, has_hi = p2 < P - 1;
            const double m = lane_below<1, DPP>(e1, lane);
            const double pp = lane_above<1, DPP>(e0, lane);
            l0 = has_lo ? m : 0.0; u0 = e1;
            l1 = e0; u1 = has_hi ? pp : 0.0;
        } else {
            const int dl = 1 << (k - 1);
            const bool has_lo = p2 >= dl, has_hi = p2 + dl < P;
            double x0, x1, y0, y1;
            switch (k) {
                case 1: fetch4<1, DPP>(e0, e1, lane, x0, x1, y0, y1); break;
                case 2: fetch4<2, DPP>(e0, e1, lane, x0, x1, y0, y1); break;
                case 3: fetch4<4, DPP>(e0, e1, lane, x0, x1, y0, y1); break;
                case 4: fetch4<8, DPP>(e0, e1, lane, x0, x1, y0, y1); break;
                case 5: fetch4<16, DPP>(e0, e1, lane, x0, x1, y0, y1); break;
                default: fetch4<32, DPP>(e0, e1, lane, x0, x1, y0, y1); break;
            }
            l0 = has_lo ? x0 : 0.0; l1 = has_lo ? x1 : 0.0;
            u0 = has_hi ? y0 : 0.0; u1 = has_hi ? y1 : 0.0;
        }
        e0 = (e0 - qa.x * l0 - qc.x * u0) * qb.x;
        e1 = (e1 - qa.y * l1 - qc.y * u1) * qb.y;
    }
}

// Stage B of the shared-operator kernels: the interface right-hand sides
// (first/last row of every partition) go through LDS to P consecutive lanes
// per system, which run the PCR steps (DPP row shifts when a system's P
// lanes lie in one row of 16, else wavefront shuffles) using the recorded
// coefficient history.  Every thread calls it; returns X_{2p} and X_{2p+1}
// of the caller's system.
// PCR_ANY: choose per launch between the two neighbour exchanges; PCR_DPP /
// PCR_SHFL: the caller guarantees P <= 16 / uses shuffles only.
enum { PCR_ANY = 0, PCR_DPP = 1, PCR_SHFL = 2 };

template <int MODE = PCR_ANY>
__device__ __forceinline__ void shared_rhs_pcr(double *XD, const double *QA, const double *QC,
                                               const double *QB, int S, int P, int P_log2, int s,
                                               int p, double df, double dl_, double &xf,
                                               double &xl) {
    const int xpitch = xd_pitch(P);
    *reinterpret_cast<double2 *>(XD + s * xpitch + 2 * p) = double2{df, dl_};
    __syncthreads();
    {
        const int tid = threadIdx.x;
        const int s2 = tid >> P_log2;
        const int p2 = tid & (P - 1);
        const int lane = tid & 63;
        double2 *q2 = reinterpret_cast<double2 *>(XD + s2 * xpitch + 2 * p2);
        const double2 e = *q2;
        double e0 = e.x, e1 = e.y;
        if constexpr (MODE == PCR_DPP) {
            rhs_pcr<true>(e0, e1, QA, QC, QB, P, p2, lane);
        } else if constexpr (MODE == PCR_SHFL) {
            rhs_pcr<false>(e0, e1, QA, QC, QB, P, p2, lane);
        } else {
            if (P <= 16)
                rhs_pcr<true>(e0, e1, QA, QC, QB, P, p2, lane);
            else
                rhs_pcr<false>(e0, e1, QA, QC, QB, P, p2, lane);
        }
        *q2 = double2{e0, e1};
    }
    __syncthreads();
    const double2 r = *reinterpret_cast<const double2 *>(XD + s * xpitch + 2 * p);
    xf = r.x;
    xl = r.y;
}

// Stage A, the right-hand-side interface PCR (Stage B) and Stage C of one
// tile on the lane's rows dv, with the tables already built; dv becomes x.
// Every thread of the block calls it.
template <typename T, int M, int MODE = PCR_ANY>
__device__ __forceinline__ void shared_solve_rows(const SharedLds &L, char *base, int S, int P,
                                                  int P_log2, int s, int p, T (&dv)[M]) {
    const PartTab<T> tab(L, base, p, M);
    const double *PT = reinterpret_cast<const double *>(base + L.part);
    const double *QA = reinterpret_cast<const double *>(base + L.qa);
    const double *QC = QA + L.nsteps * 2 * P, *QB = QC + L.nsteps * 2 * P;
    double *XD = reinterpret_cast<double *>(base + L.xd);
    // Stage A
    const T draw0 = dv[0];
    dv[1] = tab.gh[1].x * dv[1];
#pragma unroll
    for (int j = 2; j < M; ++j) {
        const auto gh = tab.gh[j];
        dv[j] = gh.x * dv[j] - gh.y * dv[j - 1];
        // table reads are hoisted at most a few rows ahead (register pressure)
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    T dt1 = T(0);
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        dt1 += tab.pi[j] * dv[j];
        if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    const double df = PT[p] * (double)draw0 - PT[P + p] * (double)dt1;
    const double dl_ = (double)dv[M - 1];
    // Stage B: right-hand-side-only PCR inside wavefronts
    double xfd, xld;
    shared_rhs_pcr<MODE>(XD, QA, QC, QB, S, P, P_log2, s, p, df, dl_, xfd, xld);
    const T xf = (T)xfd;
    // Stage C
    dv[M - 1] = (T)xld;
#pragma unroll
    for (int j = M - 2; j >= 1; --j) {
        const auto ac = tab.ac[j];
        dv[j] = dv[j] - ac.x * xf - ac.y * dv[j + 1];
        if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
    }
    dv[0] = xf;
}

// The lane's M rows of x in a strided layout (rows past the system's end
// are not written); OffT as for load_rows.
template <typename T, int M, typename OffT>
__device__ __forceinline__ void store_rows(T *x, const LaneSys &sys, int64_t rs, int r0,
                                           const T (&dv)[M]) {
    const int rows_here = rows_in(sys, r0, M);
    char *b = reinterpret_cast<char *>(x);
    const OffT step = (OffT)(rs * (int64_t)sizeof(T));
    const OffT off = (OffT)((sys.base + (int64_t)r0 * rs) * (int64_t)sizeof(T));
    if (rows_here == M) {
#pragma unroll
        for (int j = 0; j < M; ++j)
            __builtin_nontemporal_store(dv[j], reinterpret_cast<T *>(b + (off + (OffT)j * step)));
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < rows_here)
                __builtin_nontemporal_store(dv[j], reinterpret_cast<T *>(b + (off + (OffT)j * step)));
    }
}

template <typename T, int M, bool CONTIG, typename OffT>
__global__ void __launch_bounds__((shared_max_threads<T, M>()))
k_shared(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P_log2, int *err) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t n = map.n;
    const int64_t k0 = dev::xcd_tile(blockIdx.x, gridDim.x) << S_log2;
    const LaneSys sys = dev::lane_system(map, k0 + s);
    const SharedLds L = shared_layout(sizeof(T), M, P, S);

    // 1. coefficient rows, then the right-hand sides of this lane's rows (in
    //    flight while the tables are built)
    dev::RowRegs<shared_cr<M>()> cr;
    dev::rows_prefetch<T, shared_cr<M>()>(coef, n, cr);
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the right-hand sides
    T dv[M];
    T *stg = reinterpret_cast<T *>(base + shared_stage_off(L));
    TileSysLds *tsys = reinterpret_cast<TileSysLds *>(base + shared_tsys_off(L, sizeof(T), M, P, S));
    const float invR = 1.0f / (float)(P * M);
    if constexpr (!CONTIG) {
        load_rows<T, M, OffT>(d, sys, map.row_stride, r0, dv);
    } else {
        if (tid < S) {
            const LaneSys q = dev::lane_system(map, k0 + tid);
            tsys[tid].base = q.base;
            tsys[tid].nrows = q.nrows;
        }
        __syncthreads();
        dev::stage_load<T, M>(tsys, d, S, P * M, invR, dv);
    }

    // 2-3. coefficient tables and the interface PCR history
    bool bad = false;
    shared_tables<T, T, M>(coef, n, L, base, tid, s, p, P, cr, bad);
    if constexpr (!CONTIG) mask_rows<T, M>(rows_in(sys, r0, M), dv);
    if constexpr (CONTIG) {
        T ld[M];
#pragma unroll
        for (int j = 0; j < M; ++j) ld[j] = dv[j];
        dev::stage_put<T, M>(stg, tsys, T(0), S, P * M, P * M + 1, invR, s, r0, ld, dv);
    }

    // 4-6. Stage A, Stage B, Stage C; dv becomes x
    shared_solve_rows<T, M>(L, base, S, P, P_log2, s, p, dv);

    if constexpr (!CONTIG) {
        store_rows<T, M, OffT>(x, sys, map.row_stride, r0, dv);
    } else {
        dev::stage_out<T, M>(stg, tsys, x, S, P * M, P * M + 1, invR, s, r0, dv);
    }
    if (bad) atomicOr(err, 1);
}

// System of a lane in a uniform layout (fewer than 2^31 systems), stepped
// through the tiles blockIdx.x, blockIdx.x + gridDim.x, ... without a
// division per step; 32-bit state.
struct LaneWalk {
    int32_t k, s0, s1;         // system index and its two grid coordinates
    int32_t q, r;              // one step (gridDim.x * S systems) = q rows of nsys0 + r
    __device__ void init(const SysMap &m, int32_t k0, int32_t step) {
        const int32_t n0 = (int32_t)m.nsys0;
        k = k0;
        s1 = k0 / n0;
        s0 = k0 - s1 * n0;
        q = step / n0;
        r = step - q * n0;
    }
    __device__ void advance(const SysMap &m, int32_t step) {
        k += step;
        s0 += r;
        s1 += q;
        if (s0 >= (int32_t)m.nsys0) { s0 -= (int32_t)m.nsys0; ++s1; }
    }
    // the lane's system as load_rows / store_rows take it
    __device__ LaneSys sys(const SysMap &m) const {
        LaneSys l;
        l.valid = k < m.nsys;
        l.id = k;
        l.base = l.valid ? (int64_t)s0 * m.sys_stride0 + (int64_t)s1 * m.sys_stride1 : 0;
        l.nrows = l.valid ? m.n : 0;
        return l;
    }
};

// Streaming form of k_shared for uniform strided layouts: each resident
// block builds the tables once, then walks the tiles t0, t0 + gridDim.x, ...
// (t0 = blockIdx.x, or its XCD-aware image when a tile row is narrower than
// a 128-byte line) with two register sets in turn: the next
// tile's right-hand sides are loaded into one set before the tile in the
// other set is solved and stored, so loads stay in flight through its
// barriers and arithmetic.  MODE: the interface exchange (DPP when P <= 16).
template <typename T, int M, typename OffT, int MODE>
__global__ void __launch_bounds__((shared_max_threads<T, M>()))
k_shared_stream(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P_log2, int64_t ntiles,
                int *err) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t rs = map.row_stride;
    const SharedLds L = shared_layout(sizeof(T), M, P, S);
    const int32_t step = (int32_t)gridDim.x << S_log2;
    const int32_t nt = (int32_t)ntiles;
    // tile rows narrower than a 128-byte line: first tile XCD-aware
    // (dev::xcd_tile), so that at every step the blocks of one XCD hold
    // neighbouring tiles, which share lines, under one L2
    int32_t t = (int32_t)((S * (int)sizeof(T) < 128) ? dev::xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
    LaneWalk w;
    w.init(map, (t << S_log2) + s, step);
    dev::RowRegs<shared_cr<M>()> cr;
    dev::rows_prefetch<T, shared_cr<M>()>(coef, map.n, cr);
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the right-hand sides
    T va[M], vb[M];
    int64_t ba = w.sys(map).base, bb = 0;    // element offsets of the two sets' systems
    int na = (int)w.sys(map).nrows, nb = 0;  // their rows (0 past the last system)
    auto lane_of = [&](int64_t b, int nr) {
        LaneSys l;
        l.valid = nr > 0;
        l.id = 0;
        l.base = b;
        l.nrows = nr;
        return l;
    };
    load_rows<T, M, OffT>(d, lane_of(ba, na), rs, r0, va);
    bool bad = false;
    shared_tables<T, T, M>(coef, map.n, L, base, tid, s, p, P, cr, bad);
    for (;;) {
        // tile t in va; load tile t + G into vb, then solve va
        w.advance(map, step);
        {
            const LaneSys l = w.sys(map);
            bb = l.base;
            nb = (int)l.nrows;
        }
        load_rows<T, M, OffT>(d, lane_of(bb, nb), rs, r0, vb);
        __builtin_amdgcn_sched_barrier(0);
        mask_rows<T, M>(rows_in(lane_of(ba, na), r0, M), va);
        shared_solve_rows<T, M, MODE>(L, base, S, P, P_log2, s, p, va);
        store_rows<T, M, OffT>(x, lane_of(ba, na), rs, r0, va);
        t += gridDim.x;
        if (t >= nt) break;
        // tile t in vb; load tile t + G into va, then solve vb
        w.advance(map, step);
        {
            const LaneSys l = w.sys(map);
            ba = l.base;
            na = (int)l.nrows;
        }
        load_rows<T, M, OffT>(d, lane_of(ba, na), rs, r0, va);
        __builtin_amdgcn_sched_barrier(0);
        mask_rows<T, M>(rows_in(lane_of(bb, nb), r0, M), vb);
        shared_solve_rows<T, M, MODE>(L, base, S, P, P_log2, s, p, vb);
        store_rows<T, M, OffT>(x, lane_of(bb, nb), rs, r0, vb);
        t += gridDim.x;
        if (t >= nt) break;
    }
    if (bad) atomicOr(err, 1);
}

// Rolling form of the streaming kernel (kernel 6), for partitions that
// cover n exactly: one register set of right-hand sides instead of two.
// Stage C produces the rows of x from the bottom up; each row is stored at
// once and its register takes the next tile's row M-1-j, so the next tile's
// rows arrive in the order its Stage A consumes them and the register order
// of the rows alternates between tiles (FL: logical row j in register j, or
// M-1-j).  Half the registers of two sets: 24 FP64 rows per lane fit 1024
// lanes, i.e. 16 systems (128-byte tile rows) of 64 partitions at n = 1536.
template <typename T, int M>
constexpr int roll_max_threads() { return (int)sizeof(T) * M >= 256 ? 512 : 1024; }

template <typename T, int M, int MODE, int FL, typename OffT>
__device__ __forceinline__ void shared_solve_roll(const SharedLds &L, char *base, int S, int P,
                                                  int P_log2, int s, int p, T (&v)[M],
                                                  const char *db, char *xb, OffT xo, OffT no,
                                                  OffT step, bool store, bool fetch) {
    using P2 = typename PairOf<T>::type;
    auto slot = [](int j) { return FL == 1 ? M - 1 - j : j; };
    // The tables are the same for every tile: each group of four rows reads
    // them through an offset the compiler cannot see through, so the reads
    // are not hoisted out of the walk and held in registers across it.
    const int q0 = p * (M + 1);
    const P2 *GH0 = reinterpret_cast<const P2 *>(base + L.gh);
    const P2 *AC0 = reinterpret_cast<const P2 *>(base + L.ac);
    const T *PI0 = reinterpret_cast<const T *>(base + L.pi);
    const P2 *GH = GH0 + opaque(q0), *AC = AC0 + opaque(q0);
    const T *PI = PI0 + opaque(q0);
    auto rows_group = [&] {
        const int q = opaque(q0);
        GH = GH0 + q;
        AC = AC0 + q;
        PI = PI0 + q;
    };
    const double *PT = reinterpret_cast<const double *>(base + L.part);
    const double *QA = reinterpret_cast<const double *>(base + L.qa);
    const double *QC = QA + L.nsteps * 2 * P, *QB = QC + L.nsteps * 2 * P;
    double *XD = reinterpret_cast<double *>(base + L.xd);
    // Stage A
    const T draw0 = v[slot(0)];
    v[slot(1)] = GH[1].x * v[slot(1)];
#pragma unroll
    for (int j = 2; j < M; ++j) {
        if ((j & 3) == 0) rows_group();
        const P2 gh = GH[j];
        v[slot(j)] = gh.x * v[slot(j)] - gh.y * v[slot(j - 1)];
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    rows_group();
    T dt1 = T(0);
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        dt1 += PI[j] * v[slot(j)];
        if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    const double df = PT[p] * (double)draw0 - PT[P + p] * (double)dt1;
    const double dl_ = (double)v[slot(M - 1)];
    // Stage B
    double xfd, xld;
    shared_rhs_pcr<MODE>(XD, QA, QC, QB, S, P, P_log2, s, p, df, dl_, xfd, xld);
    const T xf = (T)xfd;
    // Stage C from the bottom: each row stored at once, its register refilled
    OffT xq = xo + (OffT)(M - 1) * step;
    OffT nq = no;
    T xn = (T)xld;
    if (store) __builtin_nontemporal_store(xn, reinterpret_cast<T *>(xb + xq));
    if (fetch) v[slot(M - 1)] = __builtin_nontemporal_load(reinterpret_cast<const T *>(db + nq));
#pragma unroll
    for (int j = M - 2; j >= 1; --j) {
        if (j == M - 2 || (j & 3) == 0) rows_group();
        const P2 ac = AC[j];
        T xj = v[slot(j)] - ac.x * xf - ac.y * xn;
        xj = opaque(xj);
        xq = opaque(xq - step);
        if (store) __builtin_nontemporal_store(xj, reinterpret_cast<T *>(xb + xq));
        nq = opaque(nq + step);
        if (fetch) v[slot(j)] = __builtin_nontemporal_load(reinterpret_cast<const T *>(db + nq));
        xn = xj;
        if ((j & 3) == 1) __builtin_amdgcn_sched_barrier(0);
    }
    if (store) __builtin_nontemporal_store(xf, reinterpret_cast<T *>(xb + xo));
    if (fetch) v[slot(0)] = __builtin_nontemporal_load(reinterpret_cast<const T *>(db + (nq + step)));
}

template <typename T, int M, typename OffT, int MODE>
__global__ void __launch_bounds__((roll_max_threads<T, M>()))
k_shared_roll(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P_log2, int64_t ntiles,
              int *err) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t rs = map.row_stride;
    const SharedLds L = shared_layout(sizeof(T), M, P, S);
    const int32_t step_sys = (int32_t)gridDim.x << S_log2;
    const int32_t nt = (int32_t)ntiles;
    int32_t t = (int32_t)((S * (int)sizeof(T) < 128) ? dev::xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
    LaneWalk w;
    w.init(map, (t << S_log2) + s, step_sys);
    dev::RowRegs<shared_cr<M>()> cr;
    dev::rows_prefetch<T, shared_cr<M>()>(coef, map.n, cr);
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the right-hand sides
    T v[M];
    LaneSys l = w.sys(map);
    load_rows<T, M, OffT>(d, l, rs, r0, v);
    bool bad = false;
    shared_tables<T, T, M>(coef, map.n, L, base, tid, s, p, P, cr, bad);
    // byte offsets of a lane's row 0 (a lane past the last system: system 0)
    const OffT step = (OffT)(rs * (int64_t)sizeof(T));
    auto off_of = [&](const LaneSys &q) {
        return (OffT)((q.base + (int64_t)r0 * rs) * (int64_t)sizeof(T));
    };
    bool ok = l.valid;
    OffT xo = off_of(l);
    const char *db = reinterpret_cast<const char *>(d);
    char *xb = reinterpret_cast<char *>(x);
    auto one = [&](auto layout) {
        constexpr int F = decltype(layout)::value;
        w.advance(map, step_sys);
        const LaneSys nl = w.sys(map);
        const OffT no = off_of(nl);
        const bool fetch = t + (int32_t)gridDim.x < nt;   // the block has a next tile
        shared_solve_roll<T, M, MODE, F, OffT>(L, base, S, P, P_log2, s, p, v, db, xb, xo, no, step,
                                               ok, fetch);
        ok = nl.valid;
        xo = no;
    };
    for (;;) {
        one(std::integral_constant<int, 0>{});
        t += gridDim.x;
        if (t >= nt) break;
        one(std::integral_constant<int, 1>{});
        t += gridDim.x;
        if (t >= nt) break;
    }
    if (bad) atomicOr(err, 1);
}

// The memory traffic of k_shared_stream alone: the same tile walk, lane rows
// and register double-buffering, with no tables and no arithmetic (x = d on
// every system row).  The ceiling of that access pattern, for measurement.
template <typename T, int M, typename OffT>
__global__ void __launch_bounds__((shared_max_threads<T, M>()))
k_copy_stream(SysMap map, const T *d, T *x, int S_log2, int64_t ntiles) {
    const int tid = threadIdx.x;
    const int S = 1 << S_log2;
    const int s = tid & (S - 1);
    const int r0 = (tid >> S_log2) * M;
    const int64_t rs = map.row_stride;
    const int32_t step = (int32_t)gridDim.x << S_log2;
    const int32_t nt = (int32_t)ntiles;
    // tile rows narrower than a 128-byte line: first tile XCD-aware
    // (dev::xcd_tile), so that at every step the blocks of one XCD hold
    // neighbouring tiles, which share lines, under one L2
    int32_t t = (int32_t)((S * (int)sizeof(T) < 128) ? dev::xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
    LaneWalk w;
    w.init(map, (t << S_log2) + s, step);
    T va[M], vb[M];
    LaneSys la = w.sys(map), lb;
    load_rows<T, M, OffT>(d, la, rs, r0, va);
    for (;;) {
        w.advance(map, step);
        lb = w.sys(map);
        load_rows<T, M, OffT>(d, lb, rs, r0, vb);
        __builtin_amdgcn_sched_barrier(0);
        store_rows<T, M, OffT>(x, la, rs, r0, va);
        t += gridDim.x;
        if (t >= nt) break;
        w.advance(map, step);
        la = w.sys(map);
        load_rows<T, M, OffT>(d, la, rs, r0, va);
        __builtin_amdgcn_sched_barrier(0);
        store_rows<T, M, OffT>(x, lb, rs, r0, vb);
        t += gridDim.x;
        if (t >= nt) break;
    }
}

// Streaming form for contiguous rows of consecutive systems (system k's rows
// at k*n .. k*n+n-1, fewer than 2^31 elements in all): a tile of S systems
// is one run of S*n elements, read and written with unit-stride accesses and
// transposed through LDS, where element e of the run sits at slot e + e/n.
// Each system thus owns n + 1 slots; its last one stays zero and stands for
// every identity padding row.  Elements past the run's end are replaced by
// its last element, on loads (never used) and on stores (the same value to
// the same address), so both are branch-free.  The next tile's elements are
// in flight in registers while the current one is solved and written.
// Index math below starts from dev::opaque_tid() in every phase, so that it
// is recomputed there rather than hoisted out of the tile loop and kept live
// in registers; global accesses use 32-bit byte offsets from the tile's
// (scalar) base pointer.
template <typename T>
__device__ __forceinline__ const T &at_off(const T *p, int32_t e) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) +
                                        (uint32_t)e * (uint32_t)sizeof(T));
}

template <typename T, int M>
__device__ __forceinline__ void run_load(const T *dt, int32_t tot, int nt, T (&v)[M]) {
    const int tid = dev::opaque_tid();
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int32_t e = tid + i * nt;
        v[i] = at_off(dt, e < tot ? e : tot - 1);
    }
}

// Lanes per block of k_shared_cstream: it holds a raw tile and a row tile in
// registers, and its LDS staging buffer leaves room for one block per CU in
// the usual shapes, so the register budget per lane is raised instead.
template <typename T, int M>
constexpr int cstream_max_threads() {
    return (int)sizeof(T) * M >= 256 ? 256 : ((int)sizeof(T) * M >= 128 ? 512 : 1024);
}

template <typename T, int M, int MODE>
__global__ void __launch_bounds__((cstream_max_threads<T, M>()))
k_shared_cstream(Coef coef, const T *d, T *x, int32_t n, int32_t total, int S_log2, int P_log2,
                 int32_t ntiles, int *err) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int nt = S * P;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const SharedLds L = shared_layout(sizeof(T), M, P, S);
    T *stg = reinterpret_cast<T *>(base + shared_stage_off(L));
    const int32_t run = S * n, pitch = n + 1;
    const float invn = 1.0f / (float)n;
    auto slot = [&](int32_t e) {
        int se, re;
        dev::split_elem(e, n, invn, se, re);
        return e + se;
    };
    for (int i = tid; i < S; i += nt) stg[i * pitch + n] = T(0);
    dev::RowRegs<shared_cr<M>()> cr;
    dev::rows_prefetch<T, shared_cr<M>()>(coef, n, cr);
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the right-hand sides
    int32_t t = blockIdx.x;
    int32_t tb = t * run, tot = total - tb < run ? total - tb : run;
    T ld[M], dv[M];
    run_load<T, M>(d + tb, tot, nt, ld);
    bool bad = false;
    shared_tables<T, T, M>(coef, n, L, base, tid, s, p, P, cr, bad);   // ends with a barrier
    for (;;) {
        // tile t: its elements to LDS, the lane's rows back (padding rows
        // read the zero slot)
        {
            const int q = dev::opaque_tid();
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int32_t e = q + i * nt;
                if (e < tot) stg[slot(e)] = ld[i];
                if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();
        {
            const int q = dev::opaque_tid();
            const int qs = q & (S - 1), qr = (q >> S_log2) * M;
            const T *row = stg + qs * pitch;
#pragma unroll
            for (int j = 0; j < M; ++j) dv[j] = row[qr + j < n ? qr + j : n];
        }
        // the next tile's elements go in flight
        const int32_t tn = t + (int32_t)gridDim.x;
        const int32_t tbn = tn * run, totn = total - tbn < run ? total - tbn : run;
        if (tn < ntiles) run_load<T, M>(d + tbn, totn, nt, ld);
        __builtin_amdgcn_sched_barrier(0);
        shared_solve_rows<T, M, MODE>(L, base, S, P, P_log2, s, p, dv);
        // x of tile t through LDS (every lane read its rows before the
        // barriers inside the solve); the zero slots are not written
        {
            const int q = dev::opaque_tid();
            const int qs = q & (S - 1), qr = (q >> S_log2) * M;
            T *row = stg + qs * pitch;
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (qr + j < n) row[qr + j] = dv[j];
        }
        __syncthreads();
        {
            const int q = dev::opaque_tid();
            T *xt = x + tb;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int32_t e = q + i * nt, ec = e < tot ? e : tot - 1;
                *reinterpret_cast<T *>(reinterpret_cast<char *>(xt) + (uint32_t)ec * (uint32_t)sizeof(T)) =
                    stg[slot(ec)];
                if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (tn >= ntiles) break;
        t = tn;
        tb = tbn;
        tot = totn;
        __syncthreads();   // the staging slots are read before they are rewritten
    }
    if (bad) atomicOr(err, 1);
}

// Precision form on one tile of a shared operator, the lane's FP64
// right-hand sides dv in registers (tables built as FP32, rows past the
// system's end zero): 1 + iters FP32 solves, the residual r = d - A x and
// the interface solve in FP64 (coefficient rows in LDS), corrections summed
// into xv.  Then the per-system convergence test (refine_ratio <= tol): the
// systems that miss are appended to the fallback list, and thread 0 gets the
// tile's largest ratio (0 elsewhere), which the caller folds into the state.  Every thread of the block calls it; it ends with a barrier,
// after which the interface exchange buffer is free again, except for the
// ratios thread 0 reads.
template <int M, int MODE>
__device__ __forceinline__ double refine_rows(const SharedLds &L, char *base, int S, int P,
                                            int P_log2, int s, int p, int iters, double tol,
                                            bool bad, bool valid, int64_t sys_id,
                                            RefineState *state, const double (&dv)[M],
                                            double (&xv)[M]) {
    const int tid = threadIdx.x;
    const int r0 = p * M;
    const int R = P * M;
    const double *PT = reinterpret_cast<const double *>(base + L.part);
    const double *QA = reinterpret_cast<const double *>(base + L.qa);
    const double *QC = QA + L.nsteps * 2 * P, *QB = QC + L.nsteps * 2 * P;
    double *XD = reinterpret_cast<double *>(base + L.xd);
    const double *CO = reinterpret_cast<const double *>(base + L.co);
    const int xpitch = xd_pitch(P);
    const PartTab<float> tab(L, base, p, M);
    const double K0 = PT[p], K1 = PT[P + p];
    float e[M];
    float ecur = 0.0f, eprev = 0.0f;   // largest entry of the last two corrections
#pragma unroll
    for (int j = 0; j < M; ++j) xv[j] = 0.0;
    for (int it = 0; it <= iters; ++it) {
        if (it == 0) {
#pragma unroll
            for (int j = 0; j < M; ++j) e[j] = (float)dv[j];
        } else {
            XD[s * xpitch + 2 * p] = xv[0];
            XD[s * xpitch + 2 * p + 1] = xv[M - 1];
            __syncthreads();
            const double xlo = p > 0 ? XD[s * xpitch + 2 * p - 1] : 0.0;
            const double xhi = p < P - 1 ? XD[s * xpitch + 2 * p + 2] : 0.0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int r = r0 + j;
                const double xm = j == 0 ? xlo : xv[j > 0 ? j - 1 : 0];
                const double xp = j == M - 1 ? xhi : xv[j < M - 1 ? j + 1 : M - 1];
                e[j] = (float)(dv[j] - CO[r] * xm - CO[R + r] * xv[j] - CO[2 * R + r] * xp);
            }
        }
        const float rr0 = e[0];
        e[1] = tab.gh[1].x * e[1];
#pragma unroll
        for (int j = 2; j < M; ++j) {
            const float2 gh = tab.gh[j];
            e[j] = gh.x * e[j] - gh.y * e[j - 1];
        }
        float dt1 = 0.0f;
#pragma unroll
        for (int j = 1; j <= M - 2; ++j) dt1 += tab.pi[j] * e[j];
        const double df = K0 * (double)rr0 - K1 * (double)dt1;
        double xf, xl;
        shared_rhs_pcr<MODE>(XD, QA, QC, QB, S, P, P_log2, s, p, df, (double)e[M - 1], xf, xl);
        e[M - 1] = (float)xl;
#pragma unroll
        for (int j = M - 2; j >= 1; --j) {
            const float2 ac = tab.ac[j];
            e[j] = e[j] - ac.x * (float)xf - ac.y * e[j + 1];
        }
        e[0] = (float)xf;
        eprev = ecur;
        ecur = 0.0f;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            xv[j] += (double)e[j];
            ecur = fmaxf(ecur, fabsf(e[j]));
        }
        __syncthreads();   // XD is rewritten by the next exchange
    }
    double xmax = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) xmax = fmax(xmax, fabs(xv[j]));
    if (bad) ecur = __builtin_huge_valf();
    XD[s * xpitch + 2 * p] = pack_e(ecur, eprev);
    XD[s * xpitch + 2 * p + 1] = xmax;
    // the system's id (-1 past the last system) in its spare exchange slot
    if (p == 0) XD[s * xpitch + 2 * P] = __longlong_as_double(valid ? (long long)sys_id : -1ll);
    __syncthreads();
    // lane t reads partition (t mod P) of system (t / P): the P partitions of
    // a system are P adjacent lanes of one wavefront (P divides 64), reduced
    // by butterfly shuffles; the lane of partition 0 judges the system
    {
        const int s2 = tid >> P_log2, p2 = tid & (P - 1);
        float em, ep;
        unpack_e(XD[s2 * xpitch + 2 * p2], em, ep);
        double xm = XD[s2 * xpitch + 2 * p2 + 1];
        for (int off = P >> 1; off >= 1; off >>= 1) {
            em = fmaxf(em, __shfl_xor(em, off));
            ep = fmaxf(ep, __shfl_xor(ep, off));
            xm = fmax(xm, __shfl_xor(xm, off));
        }
        const long long id = s2 < S ? __double_as_longlong(XD[s2 * xpitch + 2 * P]) : -1ll;
        const bool judge = p2 == 0 && id >= 0;
        double rel = 0.0;
        bool miss = false;
        if (judge) {
            rel = refine_ratio(state->criterion, iters, (double)em, (double)ep, xm);
            miss = !(rel <= tol);
        }
        // (blocks narrower than a wavefront: only their own lanes)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            if (off < (int)blockDim.x) rel = fmax(rel, __shfl_xor(rel, off));
        const unsigned long long ball = __ballot(miss);
        // the wavefront's largest ratio in the second spare slot of row
        // (wavefront index) -- there are at least as many rows (S) as
        // wavefronts (S*P/64) -- for thread 0 after the barrier
        if ((tid & 63) == 0) XD[(tid >> 6) * xpitch + 2 * P + 1] = rel;
        if (ball) {
            unsigned long long first = 0;
            if ((tid & 63) == 0) first = atomicAdd(&state->not_converged, (unsigned long long)__popcll(ball));
            first = __shfl(first, 0);
            if (miss) {
                const unsigned long long slot = first + __popcll(ball & __lanemask_lt());
                if (state->fallback_list && slot < (unsigned long long)state->list_capacity)
                    state->fallback_list[slot] = (int32_t)id;
            }
        }
    }
    __syncthreads();
    double rel_max = 0.0;
    if (tid == 0)
        for (int w = 0; w < ((int)blockDim.x + 63) >> 6; ++w) rel_max = fmax(rel_max, XD[w * xpitch + 2 * P + 1]);
    return rel_max;
}

// Precision form on a shared operator, one tile per block (contiguous rows
// staged through LDS, or any strided layout).
template <int M, bool CONTIG>
__global__ void __launch_bounds__((M >= 16 ? 512 : 1024))
k_shared_refine(SysMap map, Coef coef, const double *d, double *x, int S_log2, int P_log2,
                int iters, double tol, RefineState *state) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int R = P * M;
    const int64_t n = map.n;
    const int64_t k0 = dev::xcd_tile(blockIdx.x, gridDim.x) << S_log2;
    const LaneSys sys = dev::lane_system(map, k0 + s);
    const SharedLds L = shared_layout(sizeof(float), M, P, S, false);
    const int rows_here = (int)(sys.nrows - r0 < 0 ? 0 : (sys.nrows - r0 > M ? M : sys.nrows - r0));

    dev::RowRegs<shared_cr<M>()> cr;
    dev::rows_prefetch<double, shared_cr<M>()>(coef, n, cr);
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the right-hand sides
    double dv[M];
    double *stg = reinterpret_cast<double *>(base + shared_stage_off(L));
    TileSysLds *tsys = reinterpret_cast<TileSysLds *>(base + shared_tsys_off(L, 8, M, P, S));
    const float invR = 1.0f / (float)R;
    if constexpr (!CONTIG) {
        load_rows<double, M, int64_t>(d, sys, map.row_stride, r0, dv);
    } else {
        if (tid < S) {
            const LaneSys q = dev::lane_system(map, k0 + tid);
            tsys[tid].base = q.base;
            tsys[tid].nrows = q.nrows;
        }
        __syncthreads();
        dev::stage_load<double, M>(tsys, d, S, R, invR, dv);
    }
    bool bad = false;
    shared_tables<float, double, M>(coef, n, L, base, tid, s, p, P, cr, bad);
    if constexpr (!CONTIG) mask_rows<double, M>(rows_here, dv);
    if constexpr (CONTIG) {
        double ld[M];
#pragma unroll
        for (int j = 0; j < M; ++j) ld[j] = dv[j];
        dev::stage_put<double, M>(stg, tsys, 0.0, S, R, R + 1, invR, s, r0, ld, dv);
    }
    double xv[M];
    const double rel = refine_rows<M, PCR_ANY>(L, base, S, P, P_log2, s, p, iters, tol, bad,
                                               sys.valid, sys.id, state, dv, xv);
    if (tid == 0) fold_max_rel(state, rel);
    if constexpr (!CONTIG) {
        double *px = x + sys.base + (int64_t)r0 * map.row_stride;
        const int64_t rs = map.row_stride;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < rows_here) px[j * rs] = xv[j];
    } else {
        dev::stage_out<double, M>(stg, tsys, x, S, R, R + 1, invR, s, r0, xv);
    }
}

// Walking form of k_shared_refine for uniform strided layouts: as many
// workgroups as fit the device build the tables once and then take the tiles
// t0, t0 + gridDim.x, ... one at a time.  No second register set: this
// latency-bound kernel lives on occupancy (three wavefronts per SIMD, hence
// the waves-per-EU bound), so the other resident workgroups hide each tile's
// loads; measured 12% faster than one tile per workgroup on the 256^3 sweep.
template <int M, typename OffT, int MODE>
__global__ void __launch_bounds__((M >= 16 ? 512 : 1024)) __attribute__((amdgpu_waves_per_eu(3)))
k_shared_refine_walk(SysMap map, Coef coef, const double *d, double *x, int S_log2, int P_log2,
                     int32_t ntiles, int iters, double tol, RefineState *state) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t rs = map.row_stride;
    const SharedLds L = shared_layout(sizeof(float), M, P, S, false);
    const int32_t step = (int32_t)gridDim.x << S_log2;
    int32_t t = (int32_t)((S * 8 < 128) ? dev::xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
    LaneWalk w;
    w.init(map, (t << S_log2) + s, step);
    dev::RowRegs<shared_cr<M>()> cr;
    dev::rows_prefetch<double, shared_cr<M>()>(coef, map.n, cr);
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the right-hand sides
    double dv[M], xv[M];
    LaneSys la = w.sys(map);
    load_rows<double, M, OffT>(d, la, rs, r0, dv);
    bool bad = false;
    shared_tables<float, double, M>(coef, map.n, L, base, tid, s, p, P, cr, bad);
    double rel = 0.0;   // largest convergence ratio of the block's tiles (thread 0)
    for (;;) {
        mask_rows<double, M>(rows_in(la, r0, M), dv);
        rel = fmax(rel, refine_rows<M, MODE>(L, base, S, P, P_log2, s, p, iters, tol, bad, la.valid,
                                             la.id, state, dv, xv));
        store_rows<double, M, OffT>(x, la, rs, r0, xv);
        t += gridDim.x;
        if (t >= ntiles) break;
        w.advance(map, step);
        la = w.sys(map);
        load_rows<double, M, OffT>(d, la, rs, r0, dv);
        __syncthreads();   // the exchange buffers are rewritten by the next tile
    }
    if (tid == 0) fold_max_rel(state, rel);
}

// Resident blocks of a kernel on the current device.
template <typename K>
int64_t resident_blocks(K kernel, int threads, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess)
        return 0;
    return (int64_t)cus * per_cu;
}

// Largest byte offset of a uniform strided layout, to pick 32-bit offsets.
inline bool offsets_fit_32(const SysMap &m, size_t esz) {
    const int64_t nsys1 = (m.nsys + m.nsys0 - 1) / m.nsys0;
    const int64_t last = (m.n - 1) * m.row_stride + (m.nsys0 - 1) * m.sys_stride0 +
                         (nsys1 - 1) * m.sys_stride1;
    return last >= 0 && (last + 1) * (int64_t)esz <= (int64_t)0xFFFFFFFF;
}

template <typename T, int M, typename OffT, int MODE>
hipError_t launch_stream(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                         void *x, int *err, size_t lds, hipStream_t st, int64_t blocks,
                         int P_log2) {
    const int64_t resident = resident_blocks(k_shared_stream<T, M, OffT, MODE>, sh.threads(), lds);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL((k_shared_stream<T, M, OffT, MODE>), dim3((unsigned)grid), dim3(sh.threads()),
                       lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2, P_log2, blocks, err);
    return hipGetLastError();
}

template <typename T, int M, typename OffT, int MODE>
hipError_t launch_roll(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                       void *x, int *err, size_t lds, hipStream_t st, int64_t blocks, int P_log2) {
    const int64_t resident = resident_blocks(k_shared_roll<T, M, OffT, MODE>, sh.threads(), lds);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL((k_shared_roll<T, M, OffT, MODE>), dim3((unsigned)grid), dim3(sh.threads()),
                       lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2, P_log2, blocks, err);
    return hipGetLastError();
}

template <typename T, int M, typename OffT>
hipError_t launch_strided(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                          void *x, int *err, size_t lds, hipStream_t st, int64_t blocks,
                          int P_log2) {
    // the streaming form walks 32-bit system indices of a plain uniform map
    // (an index reaches at most one grid stride past the last tile, below
    // 2 * blocks * S); anything else takes the one-tile-per-block form, which
    // gives the same results
    const int64_t S = (int64_t)1 << sh.S_log2;
    const bool stream_ok = !map.offsets && !map.sys_list && !map.count &&
                           2 * (blocks + 1) * S < ((int64_t)1 << 31);
    if (sh.kernel == 6 && stream_ok && (int64_t)sh.P * M == map.n) {
        if (sh.P <= 16)
            return launch_roll<T, M, OffT, PCR_DPP>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
        return launch_roll<T, M, OffT, PCR_SHFL>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
    }
    if ((sh.kernel == 2 || sh.kernel == 6) && stream_ok && sh.threads() <= shared_max_threads<T, M>()) {
        if (sh.P <= 16)
            return launch_stream<T, M, OffT, PCR_DPP>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
        return launch_stream<T, M, OffT, PCR_SHFL>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
    } else if (sh.threads() > shared_max_threads<T, M>()) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_shared<T, M, false, OffT>), dim3((unsigned)blocks), dim3(sh.threads()),
                           lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2, P_log2, err);
    }
    return hipGetLastError();
}

// Contiguous rows of consecutive systems (system k at element k*n) with
// 32-bit element indices up to one grid stride past the last tile.
inline bool consecutive_32(const SysMap &m, int64_t S, int64_t blocks) {
    if (m.offsets || m.sys_list || m.count || m.row_stride != 1 || m.sys_stride0 != m.n) return false;
    if (m.nsys > m.nsys0 && m.sys_stride1 != m.n * m.nsys0) return false;
    return 2 * (blocks + 1) * S * m.n < ((int64_t)1 << 31);
}

template <typename T, int M, int MODE>
hipError_t launch_cstream(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                          void *x, int *err, size_t lds, hipStream_t st, int64_t blocks,
                          int P_log2) {
    const int64_t resident = resident_blocks(k_shared_cstream<T, M, MODE>, sh.threads(), lds);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL((k_shared_cstream<T, M, MODE>), dim3((unsigned)grid), dim3(sh.threads()),
                       lds, st, coef, (const T *)d, (T *)x, (int32_t)map.n,
                       (int32_t)(map.nsys * map.n), sh.S_log2, P_log2, (int32_t)blocks, err);
    return hipGetLastError();
}

template <typename T, int M>
hipError_t launch_m(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                    void *x, int *err, size_t lds, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    const int P_log2 = ilog2i(sh.P);
    if (sh.contig) {
        // the streaming form takes consecutive systems; any other contiguous
        // layout takes the one-tile-per-block form, which gives the same results
        if (sh.kernel == 2 && consecutive_32(map, S, blocks)) {
            if (sh.P <= 16)
                return launch_cstream<T, M, PCR_DPP>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
            return launch_cstream<T, M, PCR_SHFL>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
        }
        hipLaunchKernelGGL((k_shared<T, M, true, int64_t>), dim3((unsigned)blocks), dim3(sh.threads()),
                           lds, st, map, coef, (const T *)d, (T *)x, sh.S_log2, P_log2, err);
        return hipGetLastError();
    }
    if (offsets_fit_32(map, sizeof(T)))
        return launch_strided<T, M, uint32_t>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
    return launch_strided<T, M, int64_t>(map, coef, sh, d, x, err, lds, st, blocks, P_log2);
}

// The copy on the grid the streaming solve of the same shape would get
// (its resident blocks, with its LDS), so both run at the same concurrency.
template <typename T, int M, typename OffT>
hipError_t launch_copy_m(const SysMap &map, const TileShape &sh, const void *d, void *x,
                         size_t lds, hipStream_t st, int64_t blocks) {
    const int64_t resident =
        sh.P <= 16 ? resident_blocks(k_shared_stream<T, M, OffT, PCR_DPP>, sh.threads(), lds)
                   : resident_blocks(k_shared_stream<T, M, OffT, PCR_SHFL>, sh.threads(), lds);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL((k_copy_stream<T, M, OffT>), dim3((unsigned)grid), dim3(sh.threads()), 0, st,
                       map, (const T *)d, (T *)x, sh.S_log2, blocks);
    return hipGetLastError();
}

template <typename T, int M>
hipError_t launch_copy_t(const SysMap &map, const TileShape &sh, const void *d, void *x,
                         size_t lds, hipStream_t st, int64_t blocks) {
    if (offsets_fit_32(map, sizeof(T))) return launch_copy_m<T, M, uint32_t>(map, sh, d, x, lds, st, blocks);
    return launch_copy_m<T, M, int64_t>(map, sh, d, x, lds, st, blocks);
}

}  // namespace

int shared_max_threads(int dtype, int M, int kernel, bool contig) {
    const int esz = dtype == TDMA_F64 ? 8 : 4;
    if (kernel == 2 && contig) return esz * M >= 256 ? 256 : (esz * M >= 128 ? 512 : 1024);
    if (kernel == 6) return esz * M >= 256 ? 512 : 1024;
    return esz * M >= 192 ? 512 : 1024;
}

size_t shared_lds_bytes(int dtype, const TileShape &sh) {
    const int S = 1 << sh.S_log2;
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    const SharedLds L = shared_layout(esz, sh.M, sh.P, S);
    if (!sh.contig) return L.end;
    return shared_tsys_off(L, esz, sh.M, sh.P, S) + 16 * (size_t)S;
}

bool shared_supported(int dtype, const TileShape &sh) {
    if (sh.P < 1 || sh.P > 64 || (sh.P & (sh.P - 1)) != 0) return false;
    if (sh.kernel == 6 && sh.contig) return false;
    if (sh.M != 8 && sh.M != 12 && sh.M != 16 && sh.M != 24 && sh.M != 32) return false;
    if (sh.threads() > shared_max_threads(dtype, sh.M, sh.kernel, sh.contig)) return false;
    return shared_lds_bytes(dtype, sh) <= 160 * 1024;
}

bool shared_roll_ok(const SysMap &map, const TileShape &sh) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    return !sh.contig && !map.offsets && !map.sys_list && !map.count &&
           (int64_t)sh.P * sh.M == map.n && 2 * (blocks + 1) * S < ((int64_t)1 << 31);
}

hipError_t launch_shared(int dtype, const SysMap &map, const Coef &coef, const TileShape &sh,
                         const void *d, void *x, int *err, hipStream_t st) {
    const size_t lds = shared_lds_bytes(dtype, sh);
    if (dtype == TDMA_F64) {
        switch (sh.M) {
            case 8: return launch_m<double, 8>(map, coef, sh, d, x, err, lds, st);
            case 12: return launch_m<double, 12>(map, coef, sh, d, x, err, lds, st);
            case 16: return launch_m<double, 16>(map, coef, sh, d, x, err, lds, st);
            case 24: return launch_m<double, 24>(map, coef, sh, d, x, err, lds, st);
            case 32: return launch_m<double, 32>(map, coef, sh, d, x, err, lds, st);
        }
    } else if (dtype == TDMA_F32) {
        switch (sh.M) {
            case 8: return launch_m<float, 8>(map, coef, sh, d, x, err, lds, st);
            case 12: return launch_m<float, 12>(map, coef, sh, d, x, err, lds, st);
            case 16: return launch_m<float, 16>(map, coef, sh, d, x, err, lds, st);
            case 24: return launch_m<float, 24>(map, coef, sh, d, x, err, lds, st);
            case 32: return launch_m<float, 32>(map, coef, sh, d, x, err, lds, st);
        }
    }
    return hipErrorInvalidValue;
}

size_t shared_refine_lds_bytes(const TileShape &sh) {
    const int S = 1 << sh.S_log2;
    const SharedLds L = shared_layout(4, sh.M, sh.P, S, false);
    if (!sh.contig) return L.end;
    return shared_tsys_off(L, 8, sh.M, sh.P, S) + 16 * (size_t)S;
}

bool shared_refine_supported(const TileShape &sh) {
    if (sh.P < 1 || sh.P > 64 || (sh.P & (sh.P - 1)) != 0) return false;
    if (sh.M != 8 && sh.M != 16) return false;
    if (sh.threads() > (sh.M >= 16 ? 512 : 1024)) return false;
    return shared_refine_lds_bytes(sh) <= 160 * 1024;
}

hipError_t launch_shared_refine(const SysMap &map, const Coef &coef, const TileShape &sh,
                                const double *d, double *x, int iters, double tol,
                                RefineState *state, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    const size_t lds = shared_refine_lds_bytes(sh);
    const int P_log2 = ilog2i(sh.P);
    const bool walk_ok = !sh.contig && !map.offsets && !map.sys_list && !map.count &&
                         2 * (blocks + 1) * S < ((int64_t)1 << 31);
    if (walk_ok) {
        const bool o32 = offsets_fit_32(map, sizeof(double));
#define TDMA_SW(MM, OT, MD)                                                                       \
        if (sh.M == MM && o32 == std::is_same<OT, uint32_t>::value && (sh.P <= 16) == (MD == PCR_DPP)) { \
            const int64_t resident = resident_blocks(k_shared_refine_walk<MM, OT, MD>, sh.threads(), lds); \
            if (resident < 1) return hipErrorInvalidConfiguration;                                 \
            const int64_t grid = blocks < resident ? blocks : resident;                            \
            hipLaunchKernelGGL((k_shared_refine_walk<MM, OT, MD>), dim3((unsigned)grid),             \
                               dim3(sh.threads()), lds, st, map, coef, d, x, sh.S_log2, P_log2,    \
                               (int32_t)blocks, iters, tol, state);                                \
            return hipGetLastError();                                                              \
        }
        TDMA_SW(8, uint32_t, PCR_DPP) TDMA_SW(8, uint32_t, PCR_SHFL)
        TDMA_SW(8, int64_t, PCR_DPP) TDMA_SW(8, int64_t, PCR_SHFL)
        TDMA_SW(16, uint32_t, PCR_DPP) TDMA_SW(16, uint32_t, PCR_SHFL)
        TDMA_SW(16, int64_t, PCR_DPP) TDMA_SW(16, int64_t, PCR_SHFL)
#undef TDMA_SW
    }
#define TDMA_SR(MM, CT)                                                                          \
    if (sh.M == MM && sh.contig == CT) {                                                          \
        hipLaunchKernelGGL((k_shared_refine<MM, CT>), dim3((unsigned)blocks), dim3(sh.threads()), \
                           lds, st, map, coef, d, x, sh.S_log2, P_log2, iters, tol, state);      \
        return hipGetLastError();                                                                 \
    }
    TDMA_SR(8, false)
    TDMA_SR(8, true)
    TDMA_SR(16, false)
    TDMA_SR(16, true)
#undef TDMA_SR
    return hipErrorInvalidValue;
}

bool copy_streamed_supported(const SysMap &map, const TileShape &sh) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    return !sh.contig && !map.offsets && !map.sys_list && !map.count &&
           2 * (blocks + 1) * S < ((int64_t)1 << 31);
}

hipError_t launch_copy_streamed(int dtype, const SysMap &map, const TileShape &sh, const void *d,
                                void *x, hipStream_t st) {
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t blocks = (map.nsys + S - 1) / S;
    if (blocks == 0) return hipSuccess;
    if (!copy_streamed_supported(map, sh)) return hipErrorInvalidValue;
    const size_t lds = shared_lds_bytes(dtype, sh);
    if (dtype == TDMA_F64) {
        switch (sh.M) {
            case 8: return launch_copy_t<double, 8>(map, sh, d, x, lds, st, blocks);
            case 12: return launch_copy_t<double, 12>(map, sh, d, x, lds, st, blocks);
            case 16: return launch_copy_t<double, 16>(map, sh, d, x, lds, st, blocks);
            case 24: return launch_copy_t<double, 24>(map, sh, d, x, lds, st, blocks);
            case 32: return launch_copy_t<double, 32>(map, sh, d, x, lds, st, blocks);
        }
    } else if (dtype == TDMA_F32) {
        switch (sh.M) {
            case 8: return launch_copy_t<float, 8>(map, sh, d, x, lds, st, blocks);
            case 12: return launch_copy_t<float, 12>(map, sh, d, x, lds, st, blocks);
            case 16: return launch_copy_t<float, 16>(map, sh, d, x, lds, st, blocks);
            case 24: return launch_copy_t<float, 24>(map, sh, d, x, lds, st, blocks);
            case 32: return launch_copy_t<float, 32>(map, sh, d, x, lds, st, blocks);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace tdma
