// Per-row coefficients on strided layouts: every system has its own a, b, c
// beside its right-hand side d (the general batched system of Sec. 2; the
// per-row z-lines of a 3-D grid, rows 2^20 elements apart at 1024^3).
//
// Resident workgroups walk tiles of S systems x P partitions x M rows per
// lane.  S is 16 FP64 (32 FP32) systems, so every row of a tile is one
// 128-byte line and each address translation serves 128 bytes; this is what
// the one-tile-per-block kernel (S = 8, 64-byte rows) cannot reach, because
// it holds all four inputs of every row.  Here a lane keeps three values per
// interior row, alpha_j = g_j a_j, gamma_j = g_j c_j and delta_j = g_j d_j
// (g_j the pivot reciprocal of plain Thomas on the rows 1..M-2 with x_0 as a
// boundary value), computed as the rows arrive:
//  Stage A consumes the rows in order through a window of W rows whose loads
//    are in flight (row j + W is issued when row j is consumed), runs the
//    modified Thomas recurrences of tile.hip.h with O(1) running state, and
//    forms the partition's two interface rows;
//  Stage B solves the 2P-row interface systems of the tile (iface_pcr);
//  Stage C re-solves the interior from the kept values with the interface
//    unknowns as boundaries: e_j = delta_j - alpha_j e_{j-1} from e_0 = x_0,
//    then x_j = e_j - gamma_j x_{j+1} from x_{M-1}, storing each row of x
//    as it is produced.  (The same substitution as in shifted.hip, with the
//    operator rows per system instead of shared.)
// The window's registers are free from the end of Stage A, so the next
// tile's first W rows are loaded there and arrive during Stages B and C.
// 40 B per unknown in FP64 (a, b, c, d in, x out), each read or written once.
#include "tile.hip.h"
#include "walk.hip.h"

namespace tdma {
namespace {

// Lanes per workgroup: 1024 at 16 rows per lane (128 registers), 512 at 32
// (256 registers).
template <typename T, int M>
constexpr int perrow_max_threads() { return M >= 32 ? 512 : 1024; }

// Where a lane's rows are: element offsets from the kernel's array
// arguments, stepped as integers (accesses stay global-memory instructions).
template <typename T>
struct RowArrays {
    const T *a, *b, *c, *d;
};

// The 4 inputs of one row at element offset `o`.
template <typename T>
__device__ __forceinline__ void load_row(const RowArrays<T> &in, int64_t o, T &a, T &b, T &c, T &d) {
    a = __builtin_nontemporal_load(in.a + o);
    b = __builtin_nontemporal_load(in.b + o);
    c = __builtin_nontemporal_load(in.c + o);
    d = __builtin_nontemporal_load(in.d + o);
}

// Row j of a lane as the matrix has it: identity rows past the system's end
// (jl = the system's last row counted from the lane's first; FULL: every row
// is inside), no a_0 (first = the lane's partition starts the system), no
// c_{n-1}.
template <typename T, bool FULL>
__device__ __forceinline__ void fix_row(int j, int jl, bool first, T &a, T &b, T &c, T &d) {
    if (!FULL && j > jl) {
        a = T(0); b = T(1); c = T(0); d = T(0);
    }
    if (j == 0 && first) a = T(0);
    if (j == jl) c = T(0);
}

// The window of rows whose loads are in flight.
template <typename T, int W>
struct Window {
    T a[W], b[W], c[W], d[W];
};

// Element offset of row j of a partition whose row 0 is at o0: rows past the
// system's last row jl (padding) read row jl again, a valid row of the
// system even when jl < 0 (a lane wholly past the end reads the system's
// last row).
template <bool FULL>
__device__ __forceinline__ int64_t row_off(int64_t o0, int j, int jl, int64_t rs) {
    return o0 + (int64_t)(FULL || j <= jl ? j : jl) * rs;
}

// The first W rows of a partition into the window.
template <typename T, int W, bool FULL>
__device__ __forceinline__ void load_window(const RowArrays<T> &in, int64_t o0, int jl, int64_t rs,
                                            Window<T, W> &win) {
    int64_t o = opaque(row_off<FULL>(o0, 0, jl, rs));
#pragma unroll
    for (int j = 0; j < W; ++j) {
        load_row(in, o, win.a[j], win.b[j], win.c[j], win.d[j]);
        o = opaque(o + (FULL || j + 1 <= jl ? rs : 0));
    }
}

// Stage A, B and C of one tile on the lane's M rows (row 0 at o0, next
// tile's row 0 at no); the window holds rows 0..W-1 of the tile on entry
// and rows 0..W-1 of the next tile on return.  Every thread of the block
// calls it.
template <typename T, int M, int W, bool FULL, int PQ>
__device__ __forceinline__ void perrow_solve(double *XC, int S, int s, int p, int P, int P_log2,
                                             int jl, int64_t rs, const RowArrays<T> &in,
                                             Window<T, W> &win, int64_t o0, int64_t no, T *x,
                                             bool store, bool &bad) {
    static_assert(M >= 4 && W >= 1 && W < M, "a partition needs rows 0, M-1 and an interior");
    // the same for every tile: re-read through a register barrier so the
    // per-row comparisons with it are made where they are used, not hoisted
    // out of the walk and kept live across it
    if (!FULL) jl = opaque(jl);
    const bool first = p == 0;
    T al[M], ga[M], de[M];
    // rows are consumed in order; row j + W goes into the slot row j frees,
    // its offset stepped from the previous one
    int64_t lo = opaque(row_off<FULL>(o0, W, jl, rs));
    auto take = [&](int j, T &a, T &b, T &c, T &d) {
        const int sl = j % W;
        a = win.a[sl]; b = win.b[sl]; c = win.c[sl]; d = win.d[sl];
        fix_row<T, FULL>(j, jl, first, a, b, c, d);
        if (j + W < M) {
            load_row(in, lo, win.a[sl], win.b[sl], win.c[sl], win.d[sl]);
            lo = opaque(lo + (FULL || j + W + 1 <= jl ? rs : 0));
        }
    };
    T a, b, c, dd;
    // Stage A: row 0 normalised and set aside
    take(0, a, b, c, dd);
    T piv = b;
    bad |= dev::bad_pivot(piv);
    T g = dev::recip(piv);
    const T a0 = a * g, c0 = c * g, d0 = dd * g;
    // row 1: the first interior row (x_0 is a parameter)
    take(1, a, b, c, dd);
    piv = b;
    bad |= dev::bad_pivot(piv);
    g = dev::recip(piv);
    al[1] = a * g;
    ga[1] = c * g;
    de[1] = dd * g;
    T dh = de[1], ah = al[1], ch = ga[1];
    // first-row spike: x_1 = dt1 - at1 x_0 - ct1 x_{M-1} with running
    // products pi_1 = 1, pi_{j+1} = -c^_j pi_j
    T pi = T(1), dt1 = dh, at1 = ah;
#pragma unroll
    for (int j = 2; j < M; ++j) {
        take(j, a, b, c, dd);
        piv = b - a * ch;
        bad |= dev::bad_pivot(piv);
        g = dev::recip(piv);
        const T alj = a * g, gaj = c * g, dej = dd * g;
        dh = dej - alj * dh;
        ah = -alj * ah;
        pi = -ch * pi;
        ch = gaj;
        if (j <= M - 2) {
            al[j] = alj;
            ga[j] = gaj;
            de[j] = dej;
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
    // the window is free: the next tile's first rows
    load_window<T, W, FULL>(in, no, jl, rs, win);

    // Stage B
    double xfd, xld;
    iface_stage_b<PQ>(XC, S, s, p, P, P_log2, f, xfd, xld, bad);

    // Stage C, forward: e_j in place of delta_j
    const T xf = (T)xfd;
    T e = xf;
#pragma unroll
    for (int j = 1; j <= M - 2; ++j) {
        e = de[j] - al[j] * e;
        de[j] = e;
    }
    // backward: x_j, stored at once (rows j <= jl)
    int64_t xo = o0 + (int64_t)(M - 1) * rs;
    T xn = (T)xld;
    if (store && (FULL || M - 1 <= jl)) __builtin_nontemporal_store(xn, x + xo);
#pragma unroll
    for (int j = M - 2; j >= 1; --j) {
        T xj = de[j] - ga[j] * xn;
        xj = opaque(xj);
        xo = opaque(xo - rs);
        if (store && (FULL || j <= jl)) __builtin_nontemporal_store(xj, x + xo);
        xn = xj;
        if ((j & 3) == 1) __builtin_amdgcn_sched_barrier(0);
    }
    if (store && (FULL || 0 <= jl)) __builtin_nontemporal_store(xf, x + o0);
}

// Resident workgroups walk the tiles t0, t0 + G, ...; a lane past the last
// system solves a copy of system 0's rows and stores nothing.
template <typename T, int M, int W, bool FULL, int PQ>
__global__ void __launch_bounds__((perrow_max_threads<T, M>()))
k_perrow_stream(SysMap map, Coef coef, const T *d, T *x, int S_log2, int P_log2, int32_t ntiles,
                int *err) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int S = 1 << S_log2, P = 1 << P_log2;
    const int s = tid & (S - 1);
    const int p = tid >> S_log2;
    const int r0 = p * M;
    const int64_t n = map.n, rs = map.row_stride;
    const int32_t nsys0 = (int32_t)map.nsys0;
    const int32_t nsys = (int32_t)map.nsys;
    // the system's last row counted from the lane's first row (>= M - 1: all
    // M rows are inside; < 0: none is)
    const int jl = (int)(n - 1 - r0);
    RowArrays<T> in;
    in.a = (const T *)coef.a;
    in.b = (const T *)coef.b;
    in.c = (const T *)coef.c;
    in.d = d;
    const int32_t step = (int32_t)gridDim.x << S_log2;
    int32_t t = (int32_t)blockIdx.x;
    Walk w;
    w.init(nsys0, (t << S_log2) + s, step);
    auto origin = [&](const Walk &ww, bool ok) {
        return (ok ? (int64_t)ww.s0 * map.sys_stride0 + (int64_t)ww.s1 * map.sys_stride1 : 0) +
               (int64_t)r0 * rs;
    };
    bool ok = w.k < nsys;
    int64_t o0 = origin(w, ok);
    bool bad = false;
    Window<T, W> win;
    load_window<T, W, FULL>(in, o0, jl, rs, win);
    for (;;) {
        w.advance(nsys0, step);
        const bool nok = w.k < nsys;
        const int64_t no = origin(w, nok);
        bool bad_t = false;
        perrow_solve<T, M, W, FULL, PQ>(lds, S, s, p, P, P_log2, jl, rs, in, win, o0, no, x, ok, bad_t);
        bad |= bad_t && ok;
        t += gridDim.x;
        if (t >= ntiles) break;
        o0 = no;
        ok = nok;
    }
    if (bad) atomicOr(err, 1);
}

template <typename T, int M, int W, bool FULL, int PQ>
hipError_t launch_prq(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d, void *x,
                      int *err, hipStream_t st) {
    const int S = 1 << sh.S_log2;
    const int P_log2 = __builtin_ctz((unsigned)sh.P);
    const size_t lds = perrow_lds_bytes(sh);
    const int64_t ntiles = (map.nsys + S - 1) / S;
    if (ntiles == 0) return hipSuccess;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_perrow_stream<T, M, W, FULL, PQ>,
                                                         sh.threads(), lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int64_t resident = (int64_t)cus * per_cu;
    const int64_t grid = ntiles < resident ? ntiles : resident;
    hipLaunchKernelGGL((k_perrow_stream<T, M, W, FULL, PQ>), dim3((unsigned)grid), dim3(sh.threads()), lds,
                       st, map, coef, (const T *)d, (T *)x, sh.S_log2, P_log2, (int32_t)ntiles, err);
    return hipGetLastError();
}

// Stage B in its wavefront-shuffle form: the DPP form's extra registers cost
// this kernel more in spills than its shorter interface solve saves (1024^3
// per-row lines: 12.0 against 10.8 ms).
template <typename T, int M, int W, bool FULL>
hipError_t launch_pr(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d, void *x,
                     int *err, hipStream_t st) {
    return launch_prq<T, M, W, FULL, 0>(map, coef, sh, d, x, err, st);
}

template <typename T, int M, int W>
hipError_t launch_pr_full(const SysMap &map, const Coef &coef, const TileShape &sh, const void *d,
                          void *x, int *err, hipStream_t st) {
    return (int64_t)sh.P * M == map.n ? launch_pr<T, M, W, true>(map, coef, sh, d, x, err, st)
                                      : launch_pr<T, M, W, false>(map, coef, sh, d, x, err, st);
}

}  // namespace

size_t perrow_lds_bytes(const TileShape &sh) {
    return (size_t)3 * ((size_t)1 << sh.S_log2) * (2 * sh.P + 1) * sizeof(double);
}

// Kernel 5: M = 16 or 32 rows per lane, P a power of two 2..64, 1024 lanes
// (512 at 32 rows), strided uniform layouts whose walk stays in 32-bit
// system indices.
bool perrow_supported(int dtype, const TileShape &sh) {
    if (sh.kernel != 5 || sh.contig || sh.pdd) return false;
    if (dtype != TDMA_F64 && dtype != TDMA_F32) return false;
    if (sh.M != 16 && sh.M != 32) return false;
    if (sh.P < 2 || sh.P > 64 || (sh.P & (sh.P - 1)) != 0) return false;
    const int maxt = sh.M == 32 ? 512 : 1024;
    if (sh.S_log2 < 0 || sh.threads() > maxt) return false;
    return perrow_lds_bytes(sh) <= 160 * 1024;
}

bool perrow_layout_ok(const SysMap &m, const TileShape &sh) {
    if (m.offsets || m.sys_list || m.count || m.row_stride == 1) return false;
    const int64_t S = (int64_t)1 << sh.S_log2;
    const int64_t ntiles = (m.nsys + S - 1) / S;
    return 3 * (ntiles + 1) * S < ((int64_t)1 << 31);
}

hipError_t launch_perrow(int dtype, const SysMap &map, const Coef &coef, const TileShape &sh,
                         const void *d, void *x, int *err, hipStream_t st) {
    if (!perrow_supported(dtype, sh) || !perrow_layout_ok(map, sh) || coef.mode != TDMA_COEF_LIKE_D ||
        coef.shift != nullptr)
        return hipErrorInvalidValue;
    if (dtype == TDMA_F64) {
        if (sh.M == 16) return launch_pr_full<double, 16, 2>(map, coef, sh, d, x, err, st);
        return launch_pr_full<double, 32, 2>(map, coef, sh, d, x, err, st);
    }
    if (sh.M == 16) return launch_pr_full<float, 16, 4>(map, coef, sh, d, x, err, st);
    return launch_pr_full<float, 32, 4>(map, coef, sh, d, x, err, st);
}

}  // namespace tdma
