// Shared operator with a per-system diagonal shift on strided layouts: the
// FFT-Poisson z-lines of Sec. 5.2, one system per wavenumber pair, where a, b,
// c are the stretched-grid tables shared by every mode and the diagonal of
// mode k is b + shift[k] (shift = -lambda of the mode).
//
// The factors of such a system depend on its shift, so they are per system.
// What a lane keeps per row is only its right-hand side d_j and the pivot
// reciprocal g_j:
//  Stage A streams the modified Thomas recurrences of tile.hip.h over the
//    lane's M rows with O(1) running state (d^, a^, c^ of the previous row and
//    the running products of the first-row spike) and records g_j;
//  Stage B solves the 2P-row interface system (FP64 PCR inside wavefronts,
//    one system per P consecutive lanes, coefficients and right-hand sides);
//  Stage C re-solves the partition's interior rows 1..M-2 from d with the
//    interface values x_0 and x_{M-1} as known boundary values: forward
//    e_j = g_j (d_j - a_j e_{j-1}) from e_0 = x_0, backward
//    x_j = e_j - g_j c_j x_{j+1} from x_{M-1}.  From row 1 on, the pivots of
//    the modified Thomas sweep are those of plain Thomas on the interior, and
//    e_j = d^_j - a^_j x_0, so this is the substitution x = x~ - Y y of the
//    paper's Stage C written without the stored spike a^.
// Two values per row instead of the three (d^, a^, c^) of the generic fused
// kernel, so a tile of 16 FP64 systems (128-byte rows) at 32 rows per lane
// fits 512 lanes.
//
// Memory pipeline (measured on the 1024^3 Poisson lines, FP64, 16 x 32 x 32
// tiles): resident workgroups walk the tiles; each row of x is stored as soon
// as the backward pass produces it, and the register it frees is refilled at
// once with a row of the next tile's right-hand side, in the order the next
// tile's Stage A reads them (so the row order in registers alternates
// between tiles).  Loads and stores are thus spread over the pass instead of
// issued in bursts: 4.79 ms against 5.38 ms for whole-tile loads and stores,
// and 4.98 ms for a second register set filled during the interface solve
// (a set filled at the start of a tile measured 6.83 ms).
//
// Stage B is where every wave of the workgroup waits and no row moves; with
// 16 or 32 partitions it runs in its DPP form (iface_pcr_rows: neighbour rows
// as VALU operands, not LDS permutes): 4.8 -> 4.5 ms.  The width of a tile row
// then decides the rest: a copy with this walk moves 128-byte rows at 0.55 of
// HBM peak and 256-byte rows at 0.65, and a 32-system tile at 32 rows per
// lane needs the whole register file when the pivots are kept beside the
// right-hand sides.  The walk that recomputes them (kernel 7,
// shift_solve_recomp) fits 32 systems in 1024 lanes: 3.9 ms, 0.55 of peak.
#include <type_traits>

#include "refine.h"
#include "tile.hip.h"
#include "walk.hip.h"

namespace tdma {
namespace {

using dev::Iface;

template <typename T> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

__host__ __device__ inline size_t al16(size_t b) { return (b + 15) & ~(size_t)15; }

// Interior rows per segment of the pivot-recomputing solve's backward pass.
constexpr int kRecompSeg = 8;

// LDS carve-up (byte offsets): the operator's rows per partition with a pitch
// of M+1 rows (the partitions a wavefront reads at once then sit on different
// banks) as pairs AB = (a_j, b_j) and CM = (c_j, m_j), where m_j is 1 on the
// system's rows and 0 on the identity rows that pad it to P*M (the shift is
// not added there); then the interface exchange (S systems x 2P rows x (a, c,
// d), pitch 2P+1).
struct ShiftLds {
    size_t ab, cm, xc, end;
};

__host__ __device__ inline ShiftLds shift_layout(size_t esz, int M, int P, int S) {
    ShiftLds L;
    const size_t rows = (size_t)P * (M + 1) * 2 * esz;
    L.ab = 0;
    L.cm = al16(L.ab + rows);
    L.xc = al16(L.cm + rows);
    L.end = al16(L.xc + (size_t)3 * S * (2 * P + 1) * sizeof(double));
    return L;
}

// The tile's operator rows into LDS (once per workgroup), identity rows past n.
template <typename T>
__device__ __forceinline__ void build_rows(const Coef &coef, int64_t n, int M, int P, char *base,
                                           const ShiftLds &L) {
    using T2 = typename Pair2<T>::type;
    const T *A = (const T *)coef.a, *B = (const T *)coef.b, *C = (const T *)coef.c;
    T2 *AB = reinterpret_cast<T2 *>(base + L.ab);
    T2 *CM = reinterpret_cast<T2 *>(base + L.cm);
    const int R = P * M;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const bool in = r < n;
        const int p = r / M, j = r - p * M;
        const int q = p * (M + 1) + j;
        AB[q] = T2{in && r > 0 ? A[r] : T(0), in ? B[r] : T(1)};
        CM[q] = T2{in && r < n - 1 ? C[r] : T(0), in ? T(1) : T(0)};
    }
    __syncthreads();
}

// Where the x rows of a lane go and, when the walk rolls on, where the next
// tile's right-hand side rows come from.  Addresses are the kernel's array
// arguments plus element offsets: stepped through opaque() as integers, the
// accesses stay global-memory instructions (an opaque pointer would be a
// generic one, whose flat accesses also count against the LDS wait counter).
template <typename T>
struct LaneIo {
    T *x;              // the x array
    const T *d;        // the d array (ROLL)
    int64_t xo;        // row 0 of the lane's partition in x (elements)
    int64_t no;        // row 0 of the lane's partition of the next tile in d (ROLL)
    int64_t rs;        // row stride (elements)
    int nrow;          // rows of the partition inside the system (0..M)
    bool valid;        // the lane's system exists (else nothing is stored)
};

// Stage A, B and C of one tile on the lane's M rows (right-hand sides in;
// rows at or past the system's end must hold 0).  Logical row j lives in
// register slot j, or M-1-j when FL is 1.  Each row of x is stored as soon as
// the backward pass produces it; with ROLL the freed slot is refilled with
// row M-1-j of the next tile (ascending order), which puts that tile in the
// other layout (FL of the next call = 1 - FL).  Every thread of the block
// calls it.
template <typename T, int M, int FL, bool ROLL, int PQ>
__device__ __forceinline__ void shift_solve(const char *base, const ShiftLds &L, int S, int s,
                                            int p, int P, int P_log2, T sh, T (&v)[M],
                                            const LaneIo<T> &io, bool &bad) {
    static_assert(M >= 4, "a partition needs rows 0, M-1 and an interior");
    using T2 = typename Pair2<T>::type;
    auto slot = [](int j) { return FL == 1 ? M - 1 - j : j; };
    // The operator rows are the same for every tile.  Each group of four rows
    // reads them through a row offset the compiler cannot see through, so the
    // reads are neither hoisted out of the tile walk nor merged between Stage
    // A and Stage C, either of which would hold them in registers (up to
    // eight per row) across the interface solve.
    const int q0 = p * (M + 1);
    const T2 *AB0 = reinterpret_cast<const T2 *>(base + L.ab);
    const T2 *CM0 = reinterpret_cast<const T2 *>(base + L.cm);
    const T2 *AB = AB0 + opaque(q0), *CM = CM0 + opaque(q0);
    auto rows_group = [&] {
        const int q = opaque(q0);
        AB = AB0 + q;
        CM = CM0 + q;
    };
    double *XC = reinterpret_cast<double *>(const_cast<char *>(base) + L.xc);

    // Stage A: row 0 normalised and set aside, rows 1.. eliminated with x_0
    // as a parameter; g_j kept for the interior rows 1..M-2
    T g[M];
    T2 ab = AB[0], cm = CM[0];
    T piv = ab.y + cm.y * sh;
    bad |= dev::bad_pivot(piv);
    T gj = dev::recip(piv);
    const T a0 = ab.x * gj, c0 = cm.x * gj, d0 = v[slot(0)] * gj;
    ab = AB[1];
    cm = CM[1];
    piv = ab.y + cm.y * sh;
    bad |= dev::bad_pivot(piv);
    gj = dev::recip(piv);
    g[1] = gj;
    T dh = v[slot(1)] * gj, ah = ab.x * gj, ch = cm.x * gj;
    // first-row spike: x_1 = dt1 - at1 x_0 - ct1 x_{M-1} with running
    // products pi_1 = 1, pi_{j+1} = -c^_j pi_j:  dt1 = sum_{j=1}^{M-2} pi_j d^_j,
    // at1 = sum pi_j a^_j, ct1 = -pi_{M-1}
    T pi = T(1), dt1 = dh, at1 = ah;
#pragma unroll
    for (int j = 2; j < M; ++j) {
        if ((j & 3) == 0) rows_group();
        ab = AB[j];
        cm = CM[j];
        piv = (ab.y + cm.y * sh) - ab.x * ch;
        bad |= dev::bad_pivot(piv);
        gj = dev::recip(piv);
        dh = (v[slot(j)] - ab.x * dh) * gj;
        ah = -(ab.x * gj) * ah;
        pi = -ch * pi;
        ch = cm.x * gj;
        if (j <= M - 2) {
            g[j] = gj;
            dt1 += pi * dh;
            at1 += pi * ah;
        }
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    Iface f;
    {
        const double ct1 = -(double)pi;
        const double den = 1.0 - (double)c0 * (double)at1;
        bad |= dev::bad_pivot(den);
        const double rho = dev::recip(den);
        f.fa = rho * (double)a0;
        f.fc = -rho * (double)c0 * ct1;
        f.fd = rho * ((double)d0 - (double)c0 * (double)dt1);
        f.la = (double)ah;
        f.lc = (double)ch;
        f.ld = (double)dh;
    }

    // Stage B
    double xfd, xld;
    iface_stage_b<PQ>(XC, S, s, p, P, P_log2, f, xfd, xld, bad);

    // Stage C, forward: e_j in place of d_j
    const T xf = (T)xfd;
    T e = xf;
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        if ((j & 3) == 1) rows_group();
        e = (v[slot(j)] - AB[j].x * e) * g[j];
        v[slot(j)] = e;
        if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
    }
    // backward: x_j, stored at once (offset stepped just in time); with ROLL
    // the slot takes the next tile's row M-1-j
    int64_t xo = io.xo + (int64_t)(M - 1) * io.rs;
    int64_t no = io.no;
    T xn = (T)xld;
    if (io.valid && M - 1 < io.nrow) __builtin_nontemporal_store(xn, io.x + xo);
    if constexpr (ROLL) v[slot(M - 1)] = __builtin_nontemporal_load(io.d + no);
#pragma unroll
    for (int j = M - 2; j >= 1; --j) {
        if (j == M - 2 || (j & 3) == 0) rows_group();
        T xj = v[slot(j)] - (CM[j].x * g[j]) * xn;
        // computed here, row by row: not sunk into the store's branch, where
        // all rows' operator reads would be issued at once
        xj = opaque(xj);
        xo = opaque(xo - io.rs);
        if (io.valid && j < io.nrow) __builtin_nontemporal_store(xj, io.x + xo);
        if constexpr (ROLL) {
            no = opaque(no + io.rs);
            v[slot(j)] = __builtin_nontemporal_load(io.d + no);
        } else {
            v[slot(j)] = xj;
        }
        xn = xj;
        if ((j & 3) == 1) __builtin_amdgcn_sched_barrier(0);
    }
    if (io.valid && 0 < io.nrow) __builtin_nontemporal_store(xf, io.x + io.xo);
    if constexpr (ROLL)
        v[slot(0)] = __builtin_nontemporal_load(io.d + (no + io.rs));
    else
        v[slot(0)] = xf;
}

// The same solve (FP64, walk rolling on) holding one value per row: the
// right-hand side, then e_j.  The pivot reciprocals are not kept from Stage
// A but recomputed from the LDS rows and the shift: once in Stage C's forward
// pass, which also records c_j g_j at the last row of every K-row segment of
// the interior, and once more per segment in the backward pass, forward from
// the segment's checkpoint into K registers that the substitution reads in
// reverse.  Every recomputed value comes from the same operations as in
// Stage A, so the results equal shift_solve's.  Three pivot recurrences per
// row instead of one for M + M/K + K values per lane instead of 2M: at
// M = 32 a lane's rows fit the 128 registers of a 1024-lane workgroup, and a
// tile can be 32 FP64 systems (256-byte rows) wide.  The partitions cover n
// exactly, so every row is a system row (m_j = 1: the shift is added as is)
// and a row's operator reads are (a_j, b_j) and c_j, 24 of the 32 bytes.
template <int M, int FL, int K, int PQ>
__device__ __forceinline__ void shift_solve_recomp(const char *base, const ShiftLds &L, int S, int s,
                                                   int p, int P, int P_log2, double sh,
                                                   double (&v)[M], const LaneIo<double> &io,
                                                   bool &bad) {
    static_assert(M >= 4 && K >= 1, "a partition needs rows 0, M-1 and an interior");
    using T = double;
    using T2 = double2;
    auto slot = [](int j) { return FL == 1 ? M - 1 - j : j; };
    const int q0 = p * (M + 1);
    const T2 *AB0 = reinterpret_cast<const T2 *>(base + L.ab);
    const T2 *CM0 = reinterpret_cast<const T2 *>(base + L.cm);
    const T2 *AB = AB0 + opaque(q0), *CM = CM0 + opaque(q0);
    // Each group of four rows reads the operator rows through an offset that
    // the compiler takes to depend on the running value of the recurrence, so
    // the reads of later rows wait for the rows before them instead of all
    // being issued at once into registers.
    auto rows_group = [&](T dep) {
        int q = q0;
        asm volatile("" : "+v"(q) : "v"(dep));
        AB = AB0 + q;
        CM = CM0 + q;
    };
    double *XC = reinterpret_cast<double *>(const_cast<char *>(base) + L.xc);

    // Stage A: as shift_solve, keeping no pivots
    T2 ab = AB[0], cm = CM[0];
    T piv = ab.y + sh;
    bad |= dev::bad_pivot(piv);
    T gj = dev::recip(piv);
    const T a0 = ab.x * gj, c0 = cm.x * gj, d0 = v[slot(0)] * gj;
    ab = AB[1];
    cm = CM[1];
    piv = ab.y + sh;
    bad |= dev::bad_pivot(piv);
    gj = dev::recip(piv);
    T dh = v[slot(1)] * gj, ah = ab.x * gj, ch = cm.x * gj;
    T pi = T(1), dt1 = dh, at1 = ah;
#pragma unroll
    for (int j = 2; j < M; ++j) {
        if ((j & 3) == 0) rows_group(ch);
        ab = AB[j];
        cm = CM[j];
        piv = (ab.y + sh) - ab.x * ch;
        bad |= dev::bad_pivot(piv);
        gj = dev::recip(piv);
        dh = (v[slot(j)] - ab.x * dh) * gj;
        ah = -(ab.x * gj) * ah;
        pi = -ch * pi;
        ch = cm.x * gj;
        if (j <= M - 2) {
            dt1 += pi * dh;
            at1 += pi * ah;
        }
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    Iface f;
    {
        const double ct1 = -pi;
        const double den = 1.0 - c0 * at1;
        bad |= dev::bad_pivot(den);
        const double rho = dev::recip(den);
        f.fa = rho * a0;
        f.fc = -rho * c0 * ct1;
        f.fd = rho * (d0 - c0 * dt1);
        f.la = ah;
        f.lc = ch;
        f.ld = dh;
    }

    // Stage B
    double xfd, xld;
    iface_stage_b<PQ>(XC, S, s, p, P, P_log2, f, xfd, xld, bad);

    // the pivot of interior row j from c_{j-1} g_{j-1} (row 1 has none)
    auto pivot = [&](int j, T2 abj, T2 cmj, T chp) {
        return j == 1 ? abj.y + sh : (abj.y + sh) - abj.x * chp;
    };
    // Stage C, forward: e_j in place of d_j; ck[i] = c_j g_j at the last row
    // of interior segment i (rows 1 + iK .. (i+1)K)
    constexpr int NI = M - 2;
    constexpr int NSEG = (NI + K - 1) / K;
    T ck[NSEG];
    T e = xfd, chp = T(0);
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        if ((j & 3) == 1) rows_group(e);
        const T2 abj = AB[j], cmj = CM[j];
        const T g = dev::recip(pivot(j, abj, cmj, chp));
        e = (v[slot(j)] - abj.x * e) * g;
        v[slot(j)] = e;
        chp = cmj.x * g;
        if (j % K == 0) ck[j / K - 1] = chp;
        if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
    }
    // backward, one segment at a time from the last: its c_j g_j recomputed
    // forward from the checkpoint, then x_j stored at once and, the walk
    // rolling on, the register refilled with the next tile's row M-1-j
    int64_t xo = io.xo + (int64_t)(M - 1) * io.rs;
    int64_t no = io.no;
    T xn = xld;
    if (io.valid) __builtin_nontemporal_store(xn, io.x + xo);
    v[slot(M - 1)] = __builtin_nontemporal_load(io.d + no);
#pragma unroll
    for (int i = NSEG - 1; i >= 0; --i) {
        const int j0 = 1 + i * K, j1 = (i + 1) * K < M - 2 ? (i + 1) * K : M - 2;
        T chs[K];
        T c = i == 0 ? T(0) : ck[i - 1];
        rows_group(xn);
#pragma unroll
        for (int j = j0; j <= j1; ++j) {
            if (j > j0 && ((j - j0) & 3) == 0) rows_group(c);
            const T2 abj = AB[j], cmj = CM[j];
            c = cmj.x * dev::recip(pivot(j, abj, cmj, c));
            chs[j - j0] = c;
        }
#pragma unroll
        for (int j = j1; j >= j0; --j) {
            T xj = v[slot(j)] - chs[j - j0] * xn;
            xj = opaque(xj);
            xo = opaque(xo - io.rs);
            if (io.valid) __builtin_nontemporal_store(xj, io.x + xo);
            no = opaque(no + io.rs);
            v[slot(j)] = __builtin_nontemporal_load(io.d + no);
            xn = xj;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (io.valid) __builtin_nontemporal_store((T)xfd, io.x + io.xo);
    v[slot(0)] = __builtin_nontemporal_load(io.d + (no + io.rs));
}

// The lane's M rows of d (system base `sb` in elements, `valid` false past the
// last system; a lane past the last system reads the start of the array).
// The loads stop at row n-1 and the rows at or past n are zeroed.  Every
// element is read once per solve (non-temporal hint).
template <typename T, int M>
__device__ __forceinline__ void load_lane(const T *d, int64_t sb, bool valid, int64_t rs, int r0,
                                          int64_t n, T (&v)[M]) {
    const int64_t first = r0 < n - 1 ? r0 : n - 1;
    const int adv = (int)(n - 1 - first < M ? n - 1 - first : M);   // rows the pointer advances
    const T *src = d + (valid ? sb : 0) + first * rs;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        v[j] = __builtin_nontemporal_load(src);
        src += j < adv ? rs : 0;
    }
#pragma unroll
    for (int j = 0; j < M; ++j)
        if (r0 + j >= n) v[j] = T(0);
}

// Lanes per workgroup: 1024 (up to 128 registers per lane), 512 when a
// lane's M rows of one array fill 256 bytes (FP64 M = 32: up to 256).
template <typename T, int M>
constexpr int shift_max_threads() { return (int)sizeof(T) * M >= 256 ? 512 : 1024; }

// Resident workgroups walk the tiles t0, t0 + G, ... (t0 = blockIdx.x, or its
// XCD-aware image when a tile row is narrower than a 128-byte line, so that
// tiles sharing lines run under one L2).  ROLL (P*M == n): the next tile's
// right-hand sides are loaded row by row into the registers that Stage C
// frees (shift_solve), alternating the register layout between tiles;
// otherwise each tile is loaded whole at its start.  RC (FP64, ROLL): the
// solve that recomputes its pivots (shift_solve_recomp), in workgroups of up
// to 1024 lanes.
template <typename T, int M, bool ROLL, bool RC, int PQ>
__global__ void __launch_bounds__((RC ? 1024 : shift_max_threads<T, M>()))
k_shift_stream(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P_log2, int32_t ntiles,
               int *err) {
    static_assert(!RC || (ROLL && std::is_same<T, double>::value), "RC: FP64, rolling walk");
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t n = map.n, rs = map.row_stride;
    const int32_t nsys0 = (int32_t)map.nsys0;
    const int32_t nsys = (int32_t)map.nsys;
    const ShiftLds L = shift_layout(sizeof(T), M, P, S);
    const T *SH = (const T *)coef.shift;
    const int32_t step = (int32_t)gridDim.x << S_log2;
    int32_t t = (int32_t)((S * (int)sizeof(T) < 128) ? dev::xcd_tile(blockIdx.x, gridDim.x)
                                                      : blockIdx.x);
    Walk w;
    w.init(nsys0, (t << S_log2) + s, step);
    auto sbase = [&](const Walk &ww) {
        return (int64_t)ww.s0 * map.sys_stride0 + (int64_t)ww.s1 * map.sys_stride1;
    };
    const int nrow = (int)(n - r0 < 0 ? 0 : (n - r0 > M ? M : n - r0));
    bool bad = false;
    build_rows<T>(coef, n, M, P, base, L);
    T v[M];
    int64_t b = sbase(w);
    bool ok = w.k < nsys;
    T sh = SH[ok ? w.k : 0];
    load_lane<T, M>(d, b, ok, rs, r0, n, v);
    if constexpr (ROLL) {
        // one tile in layout F; the next tile's rows arrive in layout 1 - F
        auto one = [&](auto layout) {
            constexpr int F = decltype(layout)::value;
            w.advance(nsys0, step);
            const int64_t nb = sbase(w);
            const bool nok = w.k < nsys;
            const T nsh = SH[nok ? w.k : 0];   // issued before the rolled row loads
            LaneIo<T> io;
            io.x = x;
            io.d = d;
            io.xo = b + (int64_t)r0 * rs;
            io.no = (nok ? nb : 0) + (int64_t)r0 * rs;
            io.rs = rs;
            io.nrow = M;
            io.valid = ok;
            if constexpr (RC)
                shift_solve_recomp<M, F, kRecompSeg, PQ>(base, L, S, s, p, P, P_log2, sh, v, io, bad);
            else
                shift_solve<T, M, F, true, PQ>(base, L, S, s, p, P, P_log2, sh, v, io, bad);
            b = nb;
            ok = nok;
            sh = nsh;
        };
        for (;;) {
            one(std::integral_constant<int, 0>{});
            t += gridDim.x;
            if (t >= ntiles) break;
            one(std::integral_constant<int, 1>{});
            t += gridDim.x;
            if (t >= ntiles) break;
        }
    } else {
        for (;;) {
            LaneIo<T> io;
            io.x = x;
            io.d = d;
            io.xo = b + (int64_t)r0 * rs;
            io.no = 0;
            io.rs = rs;
            io.nrow = nrow;
            io.valid = ok;
            shift_solve<T, M, 0, false, PQ>(base, L, S, s, p, P, P_log2, sh, v, io, bad);
            t += gridDim.x;
            if (t >= ntiles) break;
            w.advance(nsys0, step);
            b = sbase(w);
            ok = w.k < nsys;
            sh = SH[ok ? w.k : 0];
            load_lane<T, M>(d, b, ok, rs, r0, n, v);
        }
    }
    if (bad) atomicOr(err, 1);
}

// ---------------------------------------------------------------------------
// Precision form on the shifted operator: FP64 d and x per row, FP32 pivot
// reciprocals g32 and an FP32 work row; per tile
//   x = 0, r = d;  repeat 1 + iters times:
//     solve A e = r with FP32 sweeps (Stage A / C in FP32, the interface
//     system in FP64), x += e, r = d - A x (FP64, operator rows from LDS);
// the FP32 pivots and the interface coefficients are built by the first
// solve and kept; later solves run only the right-hand-side recurrences of
// Stage A.  A system's convergence is judged from its last two corrections
// (refine_ratio) and the systems that miss tol are listed for the FP64
// fallback.  Registers per row: 2 + 2 (d, x) + 1 + 1 (g32, work).

// Second LDS part of the refinement, after the FP64 layout: FP32 copies of
// the operator rows (a, b, c, m per row, pitch M+1 per partition), then the
// lanes' FP32 pivot reciprocals (M rows x S*P lanes, lane-contiguous: the
// registers they would take are what the FP64 d and x need).
__host__ __device__ inline size_t shift_refine_lds(int M, int P, int S, size_t *f32_off,
                                                   size_t *g_off = nullptr) {
    const ShiftLds L = shift_layout(sizeof(double), M, P, S);
    *f32_off = L.end;
    const size_t g = al16(L.end + (size_t)P * (M + 1) * 4 * sizeof(float));
    if (g_off) *g_off = g;
    return al16(g + (size_t)M * S * P * sizeof(float));
}

template <int M, int PQ>
__device__ __forceinline__ double shift_refine_tile(const char *base, const ShiftLds &L,
                                                    const float4 *R32, float *G, int S, int s, int p, int P,
                                                    int P_log2, double sh, const double (&dv)[M],
                                                    double (&xv)[M], int iters, double tol,
                                                    bool valid, int64_t sys_id, RefineState *state) {
    const int tid = threadIdx.x;
    // operator rows through offsets the compiler cannot see through, renewed
    // every four rows (see shift_solve): the rows are the same in every pass
    // and every tile, and hoisted reads would hold them all in registers
    const int q0 = p * (M + 1);
    const double2 *AB0 = reinterpret_cast<const double2 *>(base + L.ab);
    const double2 *CM0 = reinterpret_cast<const double2 *>(base + L.cm);
    const double2 *AB = AB0 + opaque(q0), *CM = CM0 + opaque(q0);
    const float4 *R4 = R32 + opaque(q0);
    auto rows_group = [&] {
        const int q = opaque(q0);
        AB = AB0 + q;
        CM = CM0 + q;
        R4 = R32 + q;
    };
    double *XC = reinterpret_cast<double *>(const_cast<char *>(base) + L.xc);
    const int pitch = 2 * P + 1;
    const float shf = (float)sh;
    bool bad = false;
    float e[M];
    // this lane's pivot reciprocals in LDS: row j at G[j * lanes]
    float *GL = G + tid;
    const int lanes = (int)blockDim.x;
    auto gput = [&](int j, float v) { GL[j * lanes] = v; };
    auto gget = [&](int j) { return GL[j * lanes]; };
    // interface coefficients and first-row factors of the FP32 factorisation
    double fa = 0.0, fc = 0.0, la = 0.0, lc = 0.0, rho = 0.0;
    float g0 = 0.0f, c0h = 0.0f;
    float ecur = 0.0f, eprev = 0.0f;   // largest entry of the last two corrections
#pragma unroll
    for (int j = 0; j < M; ++j) xv[j] = 0.0;
    for (int it = 0; it <= iters; ++it) {
        if (it == 0) {
#pragma unroll
            for (int j = 0; j < M; ++j) e[j] = (float)dv[j];
        } else {
            // r = d - A x in FP64; the neighbours' outer rows through the exchange
            __syncthreads();
            XC[s * pitch + 2 * p] = xv[0];
            XC[s * pitch + 2 * p + 1] = xv[M - 1];
            __syncthreads();
            const double xlo = p > 0 ? XC[s * pitch + 2 * p - 1] : 0.0;
            const double xhi = p < P - 1 ? XC[s * pitch + 2 * p + 2] : 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if ((j & 3) == 0) rows_group();
                const double2 ab = AB[j], cm = CM[j];
                const double xm = j == 0 ? xlo : xv[j > 0 ? j - 1 : 0];
                const double xp = j == M - 1 ? xhi : xv[j < M - 1 ? j + 1 : M - 1];
                e[j] = (float)(dv[j] - ab.x * xm - (ab.y + cm.y * sh) * xv[j] - cm.x * xp);
                if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
        // Stage A (FP32): on the first pass the factorisation and the
        // interface coefficients, then the right-hand-side recurrences only
        const float r0v = e[0];
        float dh, dt1, pi = 1.0f;
        rows_group();
        if (it == 0) {
            float4 q = R4[0];
            float piv = q.y + q.w * shf;
            bad |= dev::bad_pivot(piv);
            g0 = dev::recip(piv);
            const float a0h = q.x * g0;
            c0h = q.z * g0;
            q = R4[1];
            piv = q.y + q.w * shf;
            bad |= dev::bad_pivot(piv);
            float gj = dev::recip(piv);
            gput(1, gj);
            dh = e[1] * gj;
            float ah = q.x * gj, ch = q.z * gj;
            float at1 = ah;
            dt1 = dh;
#pragma unroll
            for (int j = 2; j < M; ++j) {
                if ((j & 3) == 0) rows_group();
                q = R4[j];
                piv = (q.y + q.w * shf) - q.x * ch;
                bad |= dev::bad_pivot(piv);
                gj = dev::recip(piv);
                gput(j, gj);
                dh = (e[j] - q.x * dh) * gj;
                ah = -(q.x * gj) * ah;
                pi = -ch * pi;
                ch = q.z * gj;
                if (j <= M - 2) {
                    dt1 += pi * dh;
                    at1 += pi * ah;
                }
                if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
            const double den = 1.0 - (double)c0h * (double)at1;
            bad |= dev::bad_pivot(den);
            rho = dev::recip(den);
            fa = rho * (double)a0h;
            fc = rho * (double)c0h * (double)pi;   // -rho c^_0 ct1, ct1 = -pi_{M-1}
            la = (double)ah;
            lc = (double)ch;
        } else {
            const float g1 = gget(1);
            dh = e[1] * g1;
            dt1 = dh;
            float ch = R4[1].z * g1;
#pragma unroll
            for (int j = 2; j < M; ++j) {
                if ((j & 3) == 0) rows_group();
                const float4 q = R4[j];
                const float gj = gget(j);
                dh = (e[j] - q.x * dh) * gj;
                pi = -ch * pi;
                ch = q.z * gj;
                if (j <= M - 2) dt1 += pi * dh;
                if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
        Iface f;
        f.fa = fa;
        f.fc = fc;
        f.fd = rho * ((double)(r0v * g0) - (double)c0h * (double)dt1);
        f.la = la;
        f.lc = lc;
        f.ld = (double)dh;
        double xf, xl;
        iface_stage_b<PQ>(XC, S, s, p, P, P_log2, f, xf, xl, bad);
        // Stage C (FP32) on the correction, added to x in FP64
        const float xff = (float)xf;
        float ee = xff;
#pragma unroll
        for (int j = 1; j <= M - 2; ++j) {
            if ((j & 3) == 1) rows_group();
            ee = (e[j] - R4[j].x * ee) * gget(j);
            e[j] = ee;
            if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
        }
        e[M - 1] = (float)xl;
#pragma unroll
        for (int j = M - 2; j >= 1; --j) {
            if (j == M - 2 || (j & 3) == 0) rows_group();
            e[j] = e[j] - (R4[j].z * gget(j)) * e[j + 1];
            if ((j & 3) == 1) __builtin_amdgcn_sched_barrier(0);
        }
        e[0] = xff;
        eprev = ecur;
        ecur = 0.0f;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            xv[j] += (double)e[j];
            ecur = fmaxf(ecur, fabsf(e[j]));
        }
    }
    // convergence per system: the maxima over its P partitions (adjacent
    // lanes after the exchange, butterfly shuffles); the lane of partition 0
    // judges, misses go to the fallback list
    double xmax = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) xmax = fmax(xmax, fabs(xv[j]));
    if (bad) ecur = __builtin_huge_valf();
    __syncthreads();
    XC[s * pitch + 2 * p] = pack_e(ecur, eprev);
    XC[s * pitch + 2 * p + 1] = xmax;
    if (p == 0) XC[s * pitch + 2 * P] = __longlong_as_double(valid ? (long long)sys_id : -1ll);
    __syncthreads();
    double rel = 0.0;
    {
        const int s2 = tid >> P_log2, p2 = tid & (P - 1);
        float em, ep;
        unpack_e(XC[s2 * pitch + 2 * p2], em, ep);
        double xm = XC[s2 * pitch + 2 * p2 + 1];
        for (int off = P >> 1; off >= 1; off >>= 1) {
            em = fmaxf(em, __shfl_xor(em, off));
            ep = fmaxf(ep, __shfl_xor(ep, off));
            xm = fmax(xm, __shfl_xor(xm, off));
        }
        const long long id = __double_as_longlong(XC[s2 * pitch + 2 * P]);
        const bool judge = p2 == 0 && id >= 0;
        bool miss = false;
        if (judge) {
            rel = refine_ratio(state->criterion, iters, (double)em, (double)ep, xm);
            miss = !(rel <= tol);
        }
        const unsigned long long ball = __ballot(miss);
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
    return rel;
}

// Resident workgroups walk the tiles as k_shift_stream does; per tile the
// refinement on chip, then each row of x is stored and its register
// refilled with the next tile's row of d.  Every lane folds its largest
// ratio into the state once, at the end (one atomic per wavefront at most).
template <int M, bool FULL, int PQ>
__global__ void __launch_bounds__((shift_max_threads<double, M>()))
k_shift_refine(SysMap map, Coef coef, const double *d, double *x, int S_log2, int P_log2,
               int32_t ntiles, int iters, double tol, RefineState *state) {
    extern __shared__ double lds[];
    char *base = reinterpret_cast<char *>(lds);
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t n = map.n, rs = map.row_stride;
    const int32_t nsys0 = (int32_t)map.nsys0;
    const int32_t nsys = (int32_t)map.nsys;
    const ShiftLds L = shift_layout(sizeof(double), M, P, S);
    size_t f32_off = 0, g_off = 0;
    (void)shift_refine_lds(M, P, S, &f32_off, &g_off);
    float4 *R32 = reinterpret_cast<float4 *>(base + f32_off);
    float *G = reinterpret_cast<float *>(base + g_off);
    const double *SH = (const double *)coef.shift;
    const int32_t step = (int32_t)gridDim.x << S_log2;
    int32_t t = blockIdx.x;
    Walk w;
    w.init(nsys0, (t << S_log2) + s, step);
    auto sbase = [&](const Walk &ww) {
        return (int64_t)ww.s0 * map.sys_stride0 + (int64_t)ww.s1 * map.sys_stride1;
    };
    build_rows<double>(coef, n, M, P, base, L);
    {
        // FP32 copies of the operator rows for the sweeps
        const double2 *AB = reinterpret_cast<const double2 *>(base + L.ab);
        const double2 *CM = reinterpret_cast<const double2 *>(base + L.cm);
        for (int q = tid; q < P * (M + 1); q += blockDim.x)
            R32[q] = float4{(float)AB[q].x, (float)AB[q].y, (float)CM[q].x, (float)CM[q].y};
        __syncthreads();
    }
    const int nrow = (int)(n - r0 < 0 ? 0 : (n - r0 > M ? M : n - r0));
    double dv[M], xv[M];
    int64_t b = sbase(w);
    bool ok = w.k < nsys;
    int32_t id = w.k;
    double sh = SH[ok ? w.k : 0];
    if constexpr (FULL) {
        int64_t q = (ok ? b : 0) + (int64_t)r0 * rs;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            dv[j] = __builtin_nontemporal_load(d + q);
            q = opaque(q + rs);
        }
    } else {
        load_lane<double, M>(d, b, ok, rs, r0, n, dv);
    }
    double rel = 0.0;
    for (;;) {
        rel = fmax(rel, shift_refine_tile<M, PQ>(base, L, R32, G, S, s, p, P, P_log2, sh, dv, xv, iters, tol,
                                             ok, id, state));
        t += gridDim.x;
        const bool more = t < ntiles;
        w.advance(nsys0, step);
        const int64_t nb = sbase(w);
        const bool nok = more && w.k < nsys;
        const double nsh = SH[nok ? w.k : 0];
        // store x row by row, each freed register taking the next tile's row
        // of d (FULL: every row inside the system; otherwise the rows are
        // clamped to the system's last row and those past it zeroed)
        int64_t xq = b + (int64_t)r0 * rs;
        if constexpr (FULL) {
            int64_t nq = (nok ? nb : 0) + (int64_t)r0 * rs;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (ok) __builtin_nontemporal_store(xv[j], x + xq);
                xq = opaque(xq + rs);
                dv[j] = __builtin_nontemporal_load(d + nq);
                nq = opaque(nq + rs);
            }
        } else {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (ok && j < nrow) __builtin_nontemporal_store(xv[j], x + xq);
                xq = opaque(xq + rs);
            }
            load_lane<double, M>(d, nb, nok, rs, r0, n, dv);
        }
        if (!more) break;
        b = nb;
        ok = nok;
        id = w.k;
        sh = nsh;
    }
    if (tid == 0 || (tid & 63) == 0) fold_max_rel(state, rel);
}

template <typename K>
int64_t resident_of(K kernel, int threads, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess)
        return 0;
    return (int64_t)cus * per_cu;
}

template <typename T, int M, bool ROLL, bool RC, int PQ>
hipError_t launch_tq(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d, void *x,
                     int *err, hipStream_t st) {
    const int S = 1 << sh.S_log2;
    const int P_log2 = __builtin_ctz((unsigned)sh.P);
    const size_t lds = shift_layout(sizeof(T), M, sh.P, S).end;
    const int64_t ntiles = (map.nsys + S - 1) / S;
    if (ntiles == 0) return hipSuccess;
    const int64_t resident = resident_of(k_shift_stream<T, M, ROLL, RC, PQ>, sh.threads(), lds);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = ntiles < resident ? ntiles : resident;
    hipLaunchKernelGGL((k_shift_stream<T, M, ROLL, RC, PQ>), dim3((unsigned)grid), dim3(sh.threads()), lds,
                       st, map, coef, (const T *)d, (T *)x, sh.S_log2, P_log2, (int32_t)ntiles, err);
    return hipGetLastError();
}

// 16 and 32 partitions take the DPP form of Stage B (its partition count
// fixed at compile time), other counts the wavefront-shuffle form.
template <typename T, int M, bool ROLL, bool RC = false>
hipError_t launch_t(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d, void *x,
                    int *err, hipStream_t st) {
    switch (sh.P) {
        case 16: return launch_tq<T, M, ROLL, RC, 2>(map, coef, sh, d, x, err, st);
        case 32: return launch_tq<T, M, ROLL, RC, 4>(map, coef, sh, d, x, err, st);
    }
    return launch_tq<T, M, ROLL, RC, 0>(map, coef, sh, d, x, err, st);
}

template <typename T, int M>
hipError_t launch_m(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d, void *x,
                    int *err, hipStream_t st) {
    // kernel 3 rolls the walk on when the partitions cover n exactly; kernel 4
    // (and padded lengths) load each tile at its start; kernel 7 (FP64, P*M =
    // n) recomputes its pivots
    if constexpr (std::is_same<T, double>::value && (M == 16 || M == 32)) {
        if (sh.kernel == 7) {
            if ((int64_t)sh.P * M != map.n) return hipErrorInvalidValue;
            return launch_t<T, M, true, true>(map, coef, sh, d, x, err, st);
        }
    }
    if (sh.kernel == 7) return hipErrorInvalidValue;
    const bool roll = sh.kernel == 3 && (int64_t)sh.P * M == map.n;
    return roll ? launch_t<T, M, true>(map, coef, sh, d, x, err, st)
                : launch_t<T, M, false>(map, coef, sh, d, x, err, st);
}

template <int M, bool FULL, int PQ>
hipError_t launch_refine_q(const SysMap &map, const Coef &coef, const TileShape &sh, const double *d,
                           double *x, int iters, double tol, RefineState *state, hipStream_t st) {
    const int S = 1 << sh.S_log2;
    const int P_log2 = __builtin_ctz((unsigned)sh.P);
    size_t f32_off = 0;
    const size_t lds = shift_refine_lds(M, sh.P, S, &f32_off);
    const int64_t ntiles = (map.nsys + S - 1) / S;
    if (ntiles == 0) return hipSuccess;
    const int64_t resident = resident_of(k_shift_refine<M, FULL, PQ>, sh.threads(), lds);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = ntiles < resident ? ntiles : resident;
    hipLaunchKernelGGL((k_shift_refine<M, FULL, PQ>), dim3((unsigned)grid), dim3(sh.threads()), lds, st, map,
                       coef, d, x, sh.S_log2, P_log2, (int32_t)ntiles, iters, tol, state);
    return hipGetLastError();
}

// The precision form keeps the wavefront-shuffle Stage B: the DPP form's
// extra registers beside its FP64 d and x rows cost more in spills than the
// shorter interface solve saves (1024^3 Poisson lines: 12.3 against 11.5 ms).
template <int M, bool FULL>
hipError_t launch_refine_m(const SysMap &map, const Coef &coef, const TileShape &sh, const double *d,
                           double *x, int iters, double tol, RefineState *state, hipStream_t st) {
    return launch_refine_q<M, FULL, 0>(map, coef, sh, d, x, iters, tol, state, st);
}

}  // namespace

size_t shift_lds_bytes(int dtype, const TileShape &sh) {
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    return shift_layout(esz, sh.M, sh.P, 1 << sh.S_log2).end;
}

bool shift_supported(int dtype, const TileShape &sh) {
    if (sh.kernel != 3 && sh.kernel != 4 && sh.kernel != 7) return false;
    if (sh.contig || sh.pdd) return false;
    if (sh.P < 1 || sh.P > 64 || (sh.P & (sh.P - 1)) != 0) return false;
    if (sh.kernel == 7 && (dtype != TDMA_F64 || (sh.M != 16 && sh.M != 32))) return false;
    const int maxt = dtype == TDMA_F64 && sh.M == 32 && sh.kernel != 7 ? 512 : 1024;
    if (sh.S_log2 < 0 || sh.threads() > maxt || sh.threads() < 1) return false;
    if (dtype == TDMA_F64 && sh.M != 8 && sh.M != 16 && sh.M != 32) return false;
    if (dtype == TDMA_F32 && sh.M != 8 && sh.M != 16 && sh.M != 32) return false;
    return shift_lds_bytes(dtype, sh) <= 160 * 1024;
}

// Uniform strided layouts whose walk stays in 32-bit system indices (a lane's
// index reaches at most two grid strides past the last tile).
bool shift_layout_ok(const SysMap &m, const TileShape &sh) {
    if (m.offsets || m.sys_list || m.count || m.row_stride == 1) return false;
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t ntiles = (m.nsys + S - 1) / S;
    return 3 * (ntiles + 1) * S < ((int64_t)1 << 31);
}

// Precision form: M = 16 or 32 rows per lane, P a power of two <= 64,
// 1024 lanes (512 at M = 32), uniform strided layouts as the FP64 walk.
bool shift_refine_supported(const SysMap &m, const TileShape &sh) {
    if (sh.M != 16 && sh.M != 32) return false;
    if (sh.P < 1 || sh.P > 64 || (sh.P & (sh.P - 1)) != 0) return false;
    if (sh.S_log2 < 0 || sh.threads() > (sh.M == 32 ? 512 : 1024)) return false;
    size_t off = 0;
    if (shift_refine_lds(sh.M, sh.P, 1 << sh.S_log2, &off) > 160 * 1024) return false;
    TileShape k = sh;
    k.kernel = 3;
    return shift_layout_ok(m, k);
}

hipError_t launch_shift_refine(const SysMap &map, const Coef &coef, const TileShape &sh,
                               const double *d, double *x, int iters, double tol,
                               RefineState *state, hipStream_t st) {
    if (!shift_refine_supported(map, sh) || coef.mode != TDMA_COEF_SHARED || coef.shift == nullptr)
        return hipErrorInvalidValue;
    const bool full = (int64_t)sh.P * sh.M == map.n;
    if (sh.M == 32)
        return full ? launch_refine_m<32, true>(map, coef, sh, d, x, iters, tol, state, st)
                    : launch_refine_m<32, false>(map, coef, sh, d, x, iters, tol, state, st);
    return full ? launch_refine_m<16, true>(map, coef, sh, d, x, iters, tol, state, st)
                : launch_refine_m<16, false>(map, coef, sh, d, x, iters, tol, state, st);
}

hipError_t launch_shift(int dtype, const SysMap &map, const Coef &coef, const TileShape &sh,
                        const void *d, void *x, int *err, hipStream_t st) {
    if (!shift_supported(dtype, sh) || !shift_layout_ok(map, sh) || coef.mode != TDMA_COEF_SHARED ||
        coef.shift == nullptr)
        return hipErrorInvalidValue;
    if (dtype == TDMA_F64) {
        if (sh.M == 8) return launch_m<double, 8>(map, coef, sh, d, x, err, st);
        if (sh.M == 16) return launch_m<double, 16>(map, coef, sh, d, x, err, st);
        if (sh.M == 32) return launch_m<double, 32>(map, coef, sh, d, x, err, st);
    } else {
        if (sh.M == 8) return launch_m<float, 8>(map, coef, sh, d, x, err, st);
        if (sh.M == 16) return launch_m<float, 16>(map, coef, sh, d, x, err, st);
        if (sh.M == 32) return launch_m<float, 32>(map, coef, sh, d, x, err, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace tdma
