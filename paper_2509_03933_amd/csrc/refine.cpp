// tdma_solve_refined: planning, the FP64 fallback launch and the report.
#include <algorithm>
#include <cstring>

#include <mutex>

#include "api_internal.h"
#include "refine.h"

namespace tdma {

// Tile rule of the refinement kernel: M = 16 (else 8), P = ceil(n/M) rounded up
// to a power of two when that stays <= 64 (interface PCR inside wavefronts);
// S consecutive systems per tile as in the fused rule.
static bool default_refine_shape(int64_t n, int64_t nsys, bool contig, bool like_d, TileShape *out) {
    for (int M : {16, 8}) {
        if (like_d && M != 8) continue;
        int64_t P = (n + M - 1) / M;
        int64_t P2 = 1;
        while (P2 < P) P2 <<= 1;
        if (P2 <= 64) P = P2;
        TileShape sh;
        sh.M = M;
        sh.P = (int)P;
        sh.contig = contig;
        int S_log2 = 4;
        if (contig) {
            S_log2 = 0;
            while ((2 << S_log2) * P <= 256) ++S_log2;
        }
        while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > refine_max_threads(M)) --S_log2;
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
        sh.S_log2 = S_log2;
        while (sh.S_log2 > 0 && refine_lds_bytes(sh, like_d) > 96 * 1024) --sh.S_log2;
        if (P > 1024 || !refine_supported(sh, like_d)) continue;
        *out = sh;
        return true;
    }
    return false;
}

// Shared operator without a shift: M = 16 (else 8), P a power of two <= 64,
// S = 16 consecutive systems (128-byte FP64 rows), or 256/P for contiguous rows.
static bool default_shared_refine_shape(int64_t n, int64_t nsys, bool contig, TileShape *out) {
    for (int M : {16, 8}) {
        int P = 1;
        while ((int64_t)P * M < n) P <<= 1;
        if (P > 64) continue;
        TileShape sh;
        sh.M = M;
        sh.P = P;
        sh.contig = contig;
        int S_log2 = 4;
        if (contig) {
            S_log2 = 0;
            while ((2 << S_log2) * P <= 256) ++S_log2;
        }
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
        sh.S_log2 = S_log2;
        while (sh.S_log2 > 0 && (sh.threads() > (M >= 16 ? 512 : 1024) ||
                                 shared_refine_lds_bytes(sh) > 64 * 1024))
            --sh.S_log2;
        if (!shared_refine_supported(sh)) continue;
        *out = sh;
        return true;
    }
    return false;
}

// Shared operator with a per-system shift on a strided layout (the FFT-Poisson
// lines): M = 32 rows per lane (else 16), P a power of two <= 64 with
// P*M >= n, S = 16 consecutive systems (128-byte FP64 rows) as far as the
// lanes allow (512 at M = 32, else 1024).
static bool default_shift_refine_shape(const SysMap &map, TileShape *out) {
    for (int M : {32, 16}) {
        int64_t P = 1;
        while (P * M < map.n) P <<= 1;
        if (P > 64) continue;
        TileShape sh;
        sh.M = M;
        sh.P = (int)P;
        sh.contig = false;
        int S_log2 = 4;
        const int64_t maxt = M == 32 ? 512 : 1024;
        while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > maxt) --S_log2;
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= map.nsys) --S_log2;
        sh.S_log2 = S_log2;
        if (!shift_refine_supported(map, sh)) continue;
        *out = sh;
        return true;
    }
    return false;
}

}  // namespace tdma

using namespace tdma;

namespace tdma {

// The options of a refined call, validated.
struct RefineCall {
    int iters = 3;
    double tol = 1e-15;
    int fallback = 1;
    int criterion = 0;
};

static int refine_args(const tdma_layout *layout, const tdma_coeffs *coeffs, const double *d,
                       double *x, const tdma_refine_opts *opts, RefineCall *out) {
    int rc = validate(layout, coeffs, TDMA_F64, d, x);
    if (rc != TDMA_OK) return rc;
    if (layout->offsets) return fail(TDMA_EUNSUPPORTED, "the refined path takes uniform layouts");
    RefineCall c;
    c.iters = opts ? opts->max_iters : 3;
    c.tol = opts && opts->tol > 0.0 ? opts->tol : 1e-15;
    c.fallback = opts ? opts->fallback : 1;
    c.criterion = opts ? opts->criterion : 0;
    if (c.iters < 0 || c.iters > 3) return fail(TDMA_EINVAL, "max_iters = %d (0..3)", c.iters);
    if (c.fallback != 0 && c.fallback != 1)
        return fail(TDMA_EINVAL, "fallback = %d (0 or 1)", c.fallback);
    if (c.criterion != 0 && c.criterion != 1)
        return fail(TDMA_EINVAL, "criterion = %d (0 or 1)", c.criterion);
    // the FP64 fallback re-reads d after the refinement kernel has written x
    if (c.fallback && (const void *)x == (const void *)d)
        return fail(TDMA_EINVAL, "x aliases d: the FP64 fallback re-reads d after x is written "
                    "(solve out of place, or with fallback = 0)");
    *out = c;
    return TDMA_OK;
}

// The refinement, its fallback and its report on device state the caller
// provides: `state` (the RefineState), `list` (capacity system ids), `err`
// (the numerical error flag the fallback kernels set; cleared first when
// clear_err).  The solve's launches are those of tdma_solve_refined.
static int refined_run(const tdma_layout *layout, const tdma_coeffs *coeffs, const double *d,
                       double *x, const RefineCall &c, RefineState *state, int32_t *list,
                       int64_t capacity, int *err, bool clear_err, tdma_refine_report *report,
                       hipStream_t st) {
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (report) std::memset(report, 0, sizeof *report);
    if (nsys == 0) return TDMA_OK;
    TileShape sh;
    if (!default_refine_shape(layout->n, nsys, layout->row_stride == 1,
                              coeffs->mode == TDMA_COEF_LIKE_D, &sh))
        return fail(TDMA_EUNSUPPORTED, "n = %lld is too long for the refined path",
                    (long long)layout->n);
    hipError_t e = launch_refine_init(state, list, capacity, c.criterion, clear_err ? err : nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "refine init");
    const SysMap map = make_map(layout);
    const Coef coef = make_coef(coeffs);
    TileShape ssh;
    if (coeffs->mode == TDMA_COEF_SHARED && coeffs->b_shift == nullptr &&
        default_shared_refine_shape(layout->n, nsys, layout->row_stride == 1, &ssh))
        e = launch_shared_refine(map, coef, ssh, d, x, c.iters, c.tol, state, st);
    else if (coeffs->mode == TDMA_COEF_SHARED && coeffs->b_shift != nullptr &&
             layout->row_stride != 1 && default_shift_refine_shape(map, &ssh))
        e = launch_shift_refine(map, coef, ssh, d, x, c.iters, c.tol, state, st);
    else
        e = launch_refine(map, coef, sh, d, x, c.iters, c.tol, state, st);
    if (e != hipSuccess) return hip_fail(e, "refine launch");
    if (c.fallback) {
        TileShape fsh;
        if (!default_shape(TDMA_F64, layout->n, capacity, layout->row_stride == 1, &fsh))
            return fail(TDMA_EUNSUPPORTED, "no FP64 fallback tile for n = %lld", (long long)layout->n);
        SysMap fm = map;
        fm.nsys = capacity;
        fm.sys_list = list;
        fm.count = &state->not_converged;
        e = launch_fused(TDMA_F64, fm, coef, fsh, d, x, err, st);
        if (e != hipSuccess) return hip_fail(e, "fallback launch");
        // the systems that needed the fallback are the ill-conditioned ones:
        // two rounds of double-double residual + FP64 correction
        if (polish_partitions(layout->n) <= 512) {
            e = launch_polish(map, coef, d, x, list, &state->not_converged, capacity, 2, st);
            if (e != hipSuccess) return hip_fail(e, "fallback polish");
        }
    }
    if (!report) return TDMA_OK;
    RefineState hs;
    e = hipMemcpyAsync(&hs, state, sizeof hs, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "refine report");
    double rel;
    std::memcpy(&rel, &hs.max_rel_bits, sizeof rel);
    report->iterations = c.iters;
    report->not_converged = (int64_t)hs.not_converged;
    report->fallback_systems = c.fallback ? std::min<int64_t>((int64_t)hs.not_converged, capacity) : 0;
    report->max_rel_correction = rel;
    if (!c.fallback && hs.not_converged > 0)
        return fail(TDMA_ENOCONV, "%llu systems missed tol = %g after %d steps",
                    (unsigned long long)hs.not_converged, c.tol, c.iters);
    if ((int64_t)hs.not_converged > capacity)
        return fail(TDMA_ENOCONV, "%llu systems missed tol; only %lld were re-solved in FP64",
                    (unsigned long long)hs.not_converged, (long long)capacity);
    return TDMA_OK;
}

}  // namespace tdma

// ---------------------------------------------------------------------------
// tdma_solve_refined_noalloc: the same solve for callers that cannot allocate
// device memory.  Its device state lives in `scratch`, a file-scope array every
// device holds until the process ends: bytes [0, 128) the RefineState, [128,
// 132) the numerical error flag of its fallback, [256, ...) the fallback list
// of kNoAllocList system ids.  The array's name is a host-side stand-in: its
// device address is taken once per device, with that device current, by
// hipGetSymbolAddress, and only that address is used afterwards.

namespace tdma {
constexpr int64_t kNoAllocList = (int64_t)1 << 16;
constexpr size_t kNoAllocBytes = 256 + (size_t)kNoAllocList * sizeof(int32_t);
constexpr size_t kNoAllocErr = 128;
static_assert(sizeof(RefineState) <= kNoAllocErr, "RefineState must fit before the error flag");
}  // namespace tdma

static __device__ __align__(256) unsigned char scratch[tdma::kNoAllocBytes];

namespace tdma {

constexpr int kNoAllocDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kNoAllocDevices];

// Device address of `scratch` on the current device (looked up on the
// device's first call; no allocation).
static int noalloc_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocDevices)
        return fail(TDMA_EUNSUPPORTED, "device %d (the no-allocation path serves devices 0..%d)", dev,
                    kNoAllocDevices - 1);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(TDMA_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return TDMA_OK;
}

}  // namespace tdma

extern "C" int tdma_solve_refined_noalloc(const tdma_layout *layout, const tdma_coeffs *coeffs,
                                          const double *d, double *x, const tdma_refine_opts *opts,
                                          tdma_refine_report *report, void *stream) {
    clear_error();
    RefineCall c;
    int rc = refine_args(layout, coeffs, d, x, opts, &c);
    if (rc != TDMA_OK) return rc;
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) {
        if (report) std::memset(report, 0, sizeof *report);
        return TDMA_OK;
    }
    void *ptr = nullptr;
    rc = noalloc_scratch(&ptr);
    if (rc != TDMA_OK) return rc;
    char *base = (char *)ptr;
    const int64_t capacity = std::min<int64_t>(nsys, kNoAllocList);
    int *err = (int *)(base + kNoAllocErr);
    hipStream_t st = (hipStream_t)stream;
    rc = refined_run(layout, coeffs, d, x, c, (RefineState *)base, (int32_t *)(base + 256), capacity,
                     err, true, report, st);
    if (rc != TDMA_OK || !report) return rc;
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, err, sizeof flag, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "error flag");
    if (flag) return fail(TDMA_ESINGULAR, "the FP64 fallback met a zero or non-finite pivot");
    return TDMA_OK;
}

extern "C" int tdma_solve_refined(const tdma_layout *layout, const tdma_coeffs *coeffs,
                                  const double *d, double *x, const tdma_refine_opts *opts,
                                  tdma_refine_report *report, void *stream) {
    clear_error();
    RefineCall c;
    int rc = refine_args(layout, coeffs, d, x, opts, &c);
    if (rc != TDMA_OK) return rc;
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) {
        if (report) std::memset(report, 0, sizeof *report);
        return TDMA_OK;
    }
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const int64_t capacity = std::min<int64_t>(nsys, (int64_t)1 << 16);
    void *ws = nullptr;
    rc = ctx->workspace(3, 256 + (size_t)capacity * sizeof(int32_t), &ws);
    if (rc != TDMA_OK) return rc;
    return refined_run(layout, coeffs, d, x, c, (RefineState *)ws, (int32_t *)((char *)ws + 256),
                       capacity, ctx->d_err, false, report, (hipStream_t)stream);
}
