// Pieces shared by the walking kernels on strided layouts (shifted.hip,
// perrow.hip): the system walk of resident workgroups, the wavefront PCR of
// the interface system, and a register barrier for the compiler.
#pragma once
#include <type_traits>
#include "tile.hip.h"

namespace tdma {
namespace walk_detail {

using dev::Iface;

// System of a lane in a uniform layout (fewer than 2^31 systems) stepped by
// a fixed number of systems without a division per step.
struct Walk {
    int32_t k, s0, s1, q, r;
    __device__ void init(int32_t nsys0, int32_t k0, int32_t step) {
        k = k0;
        s1 = k0 / nsys0;
        s0 = k0 - s1 * nsys0;
        q = step / nsys0;
        r = step - q * nsys0;
    }
    __device__ void advance(int32_t nsys0, int32_t step) {
        k += step;
        s0 += r;
        s1 += q;
        if (s0 >= nsys0) { s0 -= nsys0; ++s1; }
    }
};

// One PCR elimination step on a unit-diagonal row (a, c, d) with its
// neighbours at distance h below (al, cl, dl) and above (au, cu, du);
// renormalised to unit diagonal.  Missing neighbours are zero rows.
__device__ __forceinline__ void pcr_step_row(double &a, double &c, double &d, double al, double cl,
                                             double dl, double au, double cu, double du,
                                             bool &bad) {
    const double beta = 1.0 - a * cl - c * au;
    bad |= dev::bad_pivot(beta);
    const double ib = dev::recip(beta);
    const double na = -a * al, nc = -c * cu, nd = d - a * dl - c * du;
    a = na * ib;
    c = nc * ib;
    d = nd * ib;
}

// Stage B: the interface rows of the tile's S systems go through LDS to P
// consecutive lanes per system (P a power of two <= 64), which run the PCR
// steps with wavefront shuffles; the solution comes back through LDS.  For
// a distance of two rows or more, row 2p meets only the neighbours' rows 2p
// and row 2p+1 only their rows 2p+1, so the two rows are stepped one after
// the other, which holds half the neighbour values at a time.  Every thread
// of the block calls it; returns X_{2p} and X_{2p+1} of the caller's system.
__device__ __forceinline__ void iface_pcr(double *XC, int S, int s, int p, int P, int P_log2,
                                          const Iface &f, double &x_first, double &x_last,
                                          bool &bad) {
    const int R2 = 2 * P;
    const int pitch = R2 + 1;
    double *ra = XC, *rc = XC + S * pitch, *rd = XC + 2 * S * pitch;
    __syncthreads();   // the exchange is free (previous tile done reading it)
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
        // distance 1: row 2p2 meets row 2p2-1 (lane-1) and its own row 2p2+1;
        // row 2p2+1 meets its own row 2p2 and row 2p2+2 (lane+1)
        const bool has_lo = p2 > 0, has_hi = p2 < P - 1;
        const int lo = has_lo ? lane - 1 : lane, hi = has_hi ? lane + 1 : lane;
        double am = __shfl(a1, lo), cm = __shfl(c1, lo), dm = __shfl(d1, lo);
        double ap = __shfl(a0, hi), cp = __shfl(c0, hi), dp = __shfl(d0, hi);
        if (!has_lo) { am = 0.0; cm = 0.0; dm = 0.0; }
        if (!has_hi) { ap = 0.0; cp = 0.0; dp = 0.0; }
        const double oa0 = a0, oc0 = c0, od0 = d0;
        pcr_step_row(a0, c0, d0, am, cm, dm, a1, c1, d1, bad);
        pcr_step_row(a1, c1, d1, oa0, oc0, od0, ap, cp, dp, bad);
    }
    for (int h = 2; h < R2; h <<= 1) {
        const int dl = h >> 1;          // rows 2p2+e +- h live in lanes p2 +- h/2
        const bool has_lo = p2 >= dl, has_hi = p2 + dl < P;
        const int lo = has_lo ? lane - dl : lane, hi = has_hi ? lane + dl : lane;
        {
            double la = __shfl(a0, lo), lc = __shfl(c0, lo), ld = __shfl(d0, lo);
            double ua = __shfl(a0, hi), uc = __shfl(c0, hi), ud = __shfl(d0, hi);
            if (!has_lo) { la = lc = ld = 0.0; }
            if (!has_hi) { ua = uc = ud = 0.0; }
            pcr_step_row(a0, c0, d0, la, lc, ld, ua, uc, ud, bad);
        }
        __builtin_amdgcn_sched_barrier(0);
        {
            double la = __shfl(a1, lo), lc = __shfl(c1, lo), ld = __shfl(d1, lo);
            double ua = __shfl(a1, hi), uc = __shfl(c1, hi), ud = __shfl(d1, hi);
            if (!has_lo) { la = lc = ld = 0.0; }
            if (!has_hi) { ua = uc = ud = 0.0; }
            pcr_step_row(a1, c1, d1, la, lc, ld, ua, uc, ud, bad);
        }
    }
    // each lane overwrites only its own two slots: no barrier needed before
    rd[q2] = d0;
    rd[q2 + 1] = d1;
    __syncthreads();
    x_first = rd[s * pitch + 2 * p];
    x_last = rd[s * pitch + 2 * p + 1];
}

// The value of `v` in the lane M positions lower (SHR) / higher in the
// caller's row of 16 lanes, zero when that lane lies outside the row: a DPP
// row shift, a VALU operand modifier instead of an LDS permute.
template <int M, bool SHR>
__device__ __forceinline__ double row_shift(double v) {
    static_assert(M >= 1 && M < 16, "a DPP row shift moves 1..15 lanes");
    constexpr int ctrl = (SHR ? 0x110 : 0x100) + M;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, ctrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Stage B with every system's 2P interface rows on the 16 lanes of one DPP
// row, Q = 2P/16 consecutive rows per lane (P = 8Q, Q = 2 or 4, so that the
// S*P lanes of the workgroup cover the S*16 of the PCR): the PCR steps at
// distance h take their neighbour rows from the lane itself or, across lane
// boundaries, from the lanes h/Q (at least 1) away by DPP row shifts, whose
// zero outside the row stands for the missing rows beyond the system's ends.
// Against iface_pcr (two rows per lane, wavefront shuffles), every exchange
// is a VALU operand instead of an LDS round trip, which shortens the
// interface solve that all the workgroup's waves wait on.  The rows go
// through LDS (XC, layout of iface_pcr) both ways.  Every thread of the
// block calls it; threads past S*16 idle in the PCR.  Returns X_{2p} and
// X_{2p+1} of the caller's system.
template <int Q>
__device__ __forceinline__ void iface_pcr_rows(double *XC, int S, int s, int p, const Iface &f,
                                               double &x_first, double &x_last, bool &bad) {
    static_assert(Q == 2 || Q == 4, "16 or 32 partitions");
    constexpr int P = 8 * Q, R2 = 2 * P;
    constexpr int pitch = R2 + 1;
    double *ra = XC, *rc = XC + S * pitch, *rd = XC + 2 * S * pitch;
    __syncthreads();   // the exchange is free (previous tile done reading it)
    {
        const int q = s * pitch + 2 * p;
        ra[q] = f.fa; rc[q] = f.fc; rd[q] = f.fd;
        ra[q + 1] = f.la; rc[q + 1] = f.lc; rd[q + 1] = f.ld;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int s2 = t >> 4, l = t & 15;
    if (s2 < S) {
        const int q2 = s2 * pitch + Q * l;
        double a[Q], c[Q], d[Q];
#pragma unroll
        for (int e = 0; e < Q; ++e) {
            a[e] = ra[q2 + e];
            c[e] = rc[q2 + e];
            d[e] = rd[q2 + e];
        }
        // one PCR step at distance H: row Q*l + e meets rows Q*l + e -+ H.
        // At H >= Q the neighbours are row e of the lanes H/Q away, fetched
        // just before row e is updated in place (every lane runs the same
        // instructions, so the fetch sees the old values); below Q some are
        // rows of the lane itself, taken from a copy of the old rows.
        auto step = [&](auto hc) {
            constexpr int H = decltype(hc)::value;
            if constexpr (H >= Q) {
                constexpr int L = H / Q;
#pragma unroll
                for (int e = 0; e < Q; ++e) {
                    const double al = row_shift<L, true>(a[e]), cl = row_shift<L, true>(c[e]),
                                 dl = row_shift<L, true>(d[e]);
                    const double au = row_shift<L, false>(a[e]), cu = row_shift<L, false>(c[e]),
                                 du = row_shift<L, false>(d[e]);
                    pcr_step_row(a[e], c[e], d[e], al, cl, dl, au, cu, du, bad);
                }
            } else {
                double oa[Q], oc[Q], od[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) {
                    oa[e] = a[e]; oc[e] = c[e]; od[e] = d[e];
                }
#pragma unroll
                for (int e = 0; e < Q; ++e) {
                    double al, cl, dl, au, cu, du;
                    if (e - H >= 0) {
                        al = oa[e - H]; cl = oc[e - H]; dl = od[e - H];
                    } else {
                        al = row_shift<1, true>(oa[e - H + Q]);
                        cl = row_shift<1, true>(oc[e - H + Q]);
                        dl = row_shift<1, true>(od[e - H + Q]);
                    }
                    if (e + H < Q) {
                        au = oa[e + H]; cu = oc[e + H]; du = od[e + H];
                    } else {
                        au = row_shift<1, false>(oa[e + H - Q]);
                        cu = row_shift<1, false>(oc[e + H - Q]);
                        du = row_shift<1, false>(od[e + H - Q]);
                    }
                    pcr_step_row(a[e], c[e], d[e], al, cl, dl, au, cu, du, bad);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        step(std::integral_constant<int, 1>{});
        step(std::integral_constant<int, 2>{});
        step(std::integral_constant<int, 4>{});
        step(std::integral_constant<int, 8>{});
        step(std::integral_constant<int, 16>{});
        if constexpr (R2 > 32) step(std::integral_constant<int, 32>{});
        // each lane overwrites only its own rows: no barrier needed before
#pragma unroll
        for (int e = 0; e < Q; ++e) rd[q2 + e] = d[e];
    }
    __syncthreads();
    x_first = rd[s * pitch + 2 * p];
    x_last = rd[s * pitch + 2 * p + 1];
}

// Stage B: with PQ = 2 or 4 (P = 8 PQ partitions, fixed at compile time) the
// DPP form, else iface_pcr for any P.
template <int PQ>
__device__ __forceinline__ void iface_stage_b(double *XC, int S, int s, int p, int P, int P_log2,
                                              const Iface &f, double &x_first, double &x_last,
                                              bool &bad) {
    if constexpr (PQ > 0)
        iface_pcr_rows<PQ>(XC, S, s, p, f, x_first, x_last, bad);
    else
        iface_pcr(XC, S, s, p, P, P_log2, f, x_first, x_last, bad);
}

// A value the compiler cannot see through (it is then recomputed or
// re-read where it is used instead of being kept live from an earlier point).
template <typename V>
__device__ __forceinline__ V opaque(V v) {
    asm volatile("" : "+v"(v));
    return v;
}

}  // namespace walk_detail
using namespace walk_detail;
}  // namespace tdma
