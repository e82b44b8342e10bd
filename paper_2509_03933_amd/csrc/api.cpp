// Host side of the C ABI: argument validation, per-device state, planning of
// tile shapes, dispatch, and the sticky device error flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.h"

namespace tdma {

// ---------------------------------------------------------------------------
// error state

static thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = std::string(tdma_status_string(status)) + ": " + buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(TDMA_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

// ---------------------------------------------------------------------------
// per-device state

static std::mutex g_mutex;
static std::map<int, std::unique_ptr<DeviceCtx>> g_ctx;

DeviceCtx::~DeviceCtx() { release(); }

void DeviceCtx::release() {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();   // nothing issued may still use what is freed
    for (auto &kv : ragged_cache) free_ragged_plan(&kv.second);
    ragged_cache.clear();
    for (auto &w : workspaces) (void)hipFree(w.ptr);
    workspaces.clear();
    for (auto e : events) (void)hipEventDestroy(e);
    events.clear();
    for (auto s : streams) (void)hipStreamDestroy(s);
    streams.clear();
    if (d_err) (void)hipFree(d_err);
    d_err = nullptr;
    if (cur >= 0) (void)hipSetDevice(cur);
}

int get_ctx(DeviceCtx **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_mutex);
    auto it = g_ctx.find(dev);
    if (it == g_ctx.end()) {
        auto c = std::make_unique<DeviceCtx>();
        c->dev = dev;
        e = hipMalloc(&c->d_err, 4 * sizeof(int));
        if (e != hipSuccess) return fail(TDMA_ENOMEM, "device error flag: %s", hipGetErrorString(e));
        e = hipMemset(c->d_err, 0, 4 * sizeof(int));
        if (e != hipSuccess) return hip_fail(e, "hipMemset");
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) c->num_cus = prop.multiProcessorCount;
        it = g_ctx.emplace(dev, std::move(c)).first;
    }
    *out = it->second.get();
    return TDMA_OK;
}

// Device workspace of at least `bytes`, tagged by `slot` (kept across calls).
int DeviceCtx::workspace(int slot, size_t bytes, void **out) {
    for (auto &w : workspaces) {
        if (w.slot == slot) {
            if (w.bytes >= bytes) { *out = w.ptr; return TDMA_OK; }
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
            e = hipMalloc(&w.ptr, bytes);
            if (e != hipSuccess) return fail(TDMA_ENOMEM, "workspace of %zu bytes", bytes);
            w.bytes = bytes;
            *out = w.ptr;
            return TDMA_OK;
        }
    }
    Workspace w;
    w.slot = slot;
    hipError_t e = hipMalloc(&w.ptr, bytes);
    if (e != hipSuccess) return fail(TDMA_ENOMEM, "workspace of %zu bytes", bytes);
    w.bytes = bytes;
    workspaces.push_back(w);
    *out = w.ptr;
    return TDMA_OK;
}

int DeviceCtx::get_streams(int count, hipStream_t **out) {
    while ((int)streams.size() < count) {
        hipStream_t s;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        streams.push_back(s);
    }
    *out = streams.data();
    return TDMA_OK;
}

int DeviceCtx::get_events(int count, hipEvent_t **out) {
    while ((int)events.size() < count) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        events.push_back(ev);
    }
    *out = events.data();
    return TDMA_OK;
}

// ---------------------------------------------------------------------------
// validation

int validate(const tdma_layout *L, const tdma_coeffs *C, int dtype, const void *d, const void *x) {
    if (!L) return fail(TDMA_EINVAL, "layout is NULL");
    if (!C) return fail(TDMA_EINVAL, "coeffs is NULL");
    if (dtype != TDMA_F64 && dtype != TDMA_F32) return fail(TDMA_EINVAL, "unknown dtype %d", dtype);
    if (!d || !x) return fail(TDMA_EINVAL, "d and x must be non-NULL");
    if (!C->a || !C->b || !C->c) return fail(TDMA_EINVAL, "a, b and c must be non-NULL");
    if (C->mode != TDMA_COEF_LIKE_D && C->mode != TDMA_COEF_SHARED)
        return fail(TDMA_EINVAL, "unknown coefficient mode %d", C->mode);
    if (x == C->a || x == C->b || x == C->c || (C->b_shift && x == C->b_shift))
        return fail(TDMA_EINVAL, "x must not alias the coefficients");
    if (L->nsys0 < 0 || L->nsys1 < 0) return fail(TDMA_EINVAL, "negative system count");
    if (L->nsys1 > 0 && L->nsys0 > INT64_MAX / L->nsys1) return fail(TDMA_EINVAL, "nsys overflows");
    // one workgroup at most per system and 32-bit system indices in the
    // streaming kernels: a call takes fewer than 2^31 systems
    if (L->nsys0 * L->nsys1 > (int64_t)0x7fffffff)
        return fail(TDMA_EUNSUPPORTED, "%lld systems in one call (at most 2^31 - 1; split the batch)",
                    (long long)(L->nsys0 * L->nsys1));
    if (L->offsets) {
        if (L->nsys1 != 1) return fail(TDMA_EINVAL, "ragged layout needs nsys1 == 1");
        if (C->mode != TDMA_COEF_LIKE_D)
            return fail(TDMA_EINVAL, "ragged layout needs per-row (LIKE_D) coefficients");
        for (int64_t k = 0; k < L->nsys0; ++k) {
            const int64_t len = L->offsets[k + 1] - L->offsets[k];
            if (len < 2) return fail(TDMA_EINVAL, "ragged system %lld has %lld rows (< 2)",
                                     (long long)k, (long long)len);
            if (len > kMaxRaggedRows)
                return fail(TDMA_EUNSUPPORTED, "ragged system %lld has %lld rows (> %lld)",
                            (long long)k, (long long)len, (long long)kMaxRaggedRows);
        }
        if (L->offsets[0] < 0) return fail(TDMA_EINVAL, "negative offset");
        return TDMA_OK;
    }
    if (L->nsys0 * L->nsys1 == 0) return TDMA_OK;
    if (L->n < 2) return fail(TDMA_EINVAL, "n = %lld (< 2)", (long long)L->n);
    if (L->row_stride == 0 && L->n > 1) return fail(TDMA_EINVAL, "row_stride is 0");
    if (L->row_stride < 0 || L->sys_stride0 < 0 || L->sys_stride1 < 0)
        return fail(TDMA_EINVAL, "negative stride");
    // the last element any system reaches, in 128-bit arithmetic: device
    // index math is 64-bit, so the layout must span fewer than 2^62 elements
    const __int128 last = (__int128)(L->n - 1) * L->row_stride +
                          (__int128)(L->nsys0 - 1) * L->sys_stride0 +
                          (__int128)(L->nsys1 - 1) * L->sys_stride1;
    if (last >= ((__int128)1 << 62))
        return fail(TDMA_EINVAL, "the layout spans more than 2^62 elements");
    return TDMA_OK;
}

// ---------------------------------------------------------------------------
// planning of the fused path

static int ilog2_floor(int64_t v) {
    int r = 0;
    while ((int64_t)1 << (r + 1) <= v) ++r;
    return r;
}

// Built-in tile rule for uniform layouts (the autotune cache overrides it).
// Strided systems: S consecutive systems per tile so that each row load is a
// full 128-byte line (S = 16 in FP64, 32 in FP32); P partitions of M rows so
// that P*M covers n.  Contiguous rows: the tile is staged through LDS.
// Small problems (fewer than 2^20 unknowns) are latency-bound: short
// partitions (M = 4 first) and one system per tile, so the solve spreads
// over as many CUs as it can and each lane's serial chain is short.
bool default_shape(int dtype, int64_t n, int64_t nsys, bool contig, TileShape *out) {
    const int esz = dtype == TDMA_F64 ? 8 : 4;
    const bool small = n * nsys < ((int64_t)1 << 20);
    const int Ms_f64[] = {16, 8, 4};
    const int Ms_f32[] = {16, 32, 8, 4};
    const int Ms_small[] = {4, 8, 16};
    const int *Ms = small ? Ms_small : (dtype == TDMA_F64 ? Ms_f64 : Ms_f32);
    const int nM = small ? 3 : (dtype == TDMA_F64 ? 3 : 4);
    for (int mi = 0; mi < nM; ++mi) {
        const int M = Ms[mi];
        const int64_t P = (n + M - 1) / M;
        if (P > 1024) continue;
        TileShape sh;
        sh.M = M;
        sh.P = (int)P;
        sh.contig = contig;
        int S_log2 = contig ? ilog2_floor(std::max<int64_t>(1, 256 / P)) : ilog2_floor(128 / esz);
        const int maxt = fused_max_threads(dtype, M);
        while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > maxt) --S_log2;
        // a tile larger than the number of systems only wastes lanes
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
        if (small) S_log2 = 0;
        sh.S_log2 = S_log2;
        if (((int64_t)1 << S_log2) * P > maxt) continue;
        if (contig && fused_lds_bytes(dtype, sh) > 96 * 1024) continue;
        *out = sh;
        return true;
    }
    return false;
}

// Shared-operator kernel, streaming form: P a power of two <= 64 (one
// system's interface rows fit one wavefront), M rows per lane from
// {16, 32, 8, 12, 24}, the one that pads the system least (P*M - n; 12 and
// 24 fit the 3*2^k lengths exactly, measured 5-16% faster than padding them
// to 16 or 32); on ties, for strided layouts the one with at most 16
// partitions (whose interface exchange is DPP row shifts; y-lines of
// n = 512: 32 rows x 16 partitions 1.84 ms, 16 x 32 1.97-1.99 ms), then the
// earlier in that order, for contiguous rows the larger M (fewer
// partitions).  Strided layouts take
// S = 32 systems per tile (measured best on the 256^3 ADI sweep in FP64 and
// FP32), contiguous rows S = 16 and at least 256 lanes; both as far as the
// lanes and LDS allow.  Contiguous x-lines of n = 768 (FP64): 24 rows x 32
// partitions x 16 systems 1.94 ms, 12 x 64 x 8 2.26 ms, 24 x 32 x 8 2.68 ms;
// n = 384: 24 x 16 x 16 0.248 ms, 12 x 32 x 8 0.279 ms.  A streaming
// block holds its CU's LDS for the whole launch, so the whole 160 KB is
// available to it.  allow_roll admits the rolling form (kernel 6) below; the
// streamed copy keeps the two-set shape, whose lane bound its kernel shares.
bool default_shared_shape(int dtype, int64_t n, int64_t nsys, bool contig, TileShape *out,
                          bool allow_roll) {
    const int Ms[] = {16, 32, 8, 12, 24};
    bool found = false;
    TileShape best;
    for (int M : Ms) {
        int64_t P = 1;
        while (P * M < n) P <<= 1;
        if (P > 64) continue;
        TileShape sh;
        sh.kernel = 2;
        sh.M = M;
        sh.P = (int)P;
        sh.contig = contig;
        int S_log2 = contig ? ilog2_floor(std::max<int64_t>(16, 256 / P)) : 5;
        const int maxt = shared_max_threads(dtype, M, sh.kernel, contig);
        while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > maxt) --S_log2;
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
        sh.S_log2 = S_log2;
        while (sh.S_log2 > 0 && shared_lds_bytes(dtype, sh) > 160 * 1024) --sh.S_log2;
        if (!shared_supported(dtype, sh)) continue;
        const int64_t pad = (int64_t)sh.P * sh.M, best_pad = found ? (int64_t)best.P * best.M : 0;
        const bool tie_wins = contig ? sh.M > best.M : (sh.P <= 16 && best.P > 16);
        if (!found || pad < best_pad || (pad == best_pad && tie_wins)) {
            best = sh;
            found = true;
        }
    }
    // Strided rows whose two-set streaming tile is narrower than a 128-byte
    // line (its lanes are capped where M rows fill 192 bytes: the 1536-row
    // z-lines of the large sweeps take 8 systems), with partitions that cover
    // n exactly: the rolling form holds one register set and fits the full
    // 128-byte width (z-lines of 1536 rows: 3.24 -> 2.44 ms).
    const int esz = dtype == TDMA_F64 ? 8 : 4;
    if (found && allow_roll && !contig && (int64_t)best.P * best.M == n &&
        ((int64_t)esz << best.S_log2) < 128) {
        TileShape r = best;
        r.kernel = 6;
        r.S_log2 = ilog2_floor(128 / esz);
        const int maxt = shared_max_threads(dtype, r.M, 6, false);
        while (r.S_log2 > 0 && ((int64_t)1 << r.S_log2) * r.P > maxt) --r.S_log2;
        while (r.S_log2 > 0 && ((int64_t)1 << (r.S_log2 - 1)) >= nsys) --r.S_log2;
        while (r.S_log2 > 0 && shared_lds_bytes(dtype, r) > 160 * 1024) --r.S_log2;
        if (r.S_log2 > best.S_log2 && shared_supported(dtype, r)) best = r;
    }
    if (found) *out = best;
    return found;
}

// Shared operator with a per-system shift on a strided layout (the
// FFT-Poisson lines): M = 32 rows per lane (else 16, 8), P a power of two
// <= 64 with P*M >= n, and S = 16 consecutive systems per tile in FP64, 32 in
// FP32 (128-byte tile rows), as far as the lanes allow (512 for FP64 at
// M = 32, else 1024); the rolling walk (kernel 3).  In FP64 with 32 rows per
// lane and 16 or 32 partitions covering n, the walk that recomputes its
// pivots (kernel 7) with S = 32 (256-byte rows).  Measured on the 1024^3
// Poisson lines in FP64: kernel 7 with 32 x 32 partitions x 32 rows 3.9 ms;
// kernel 3 with 16 x 32 x 32 4.5 ms, 16 x 64 x 16 6.0 ms, 8 x 32 x 32 7.3 ms;
// on 1024^2 x 512 lines kernel 7 with 32 x 16 x 32 1.87 ms, kernel 3 with
// 16 x 16 x 32 2.54 ms.
static bool default_shift_shape(int dtype, int64_t n, int64_t nsys, TileShape *out) {
    const int Ms[] = {32, 16, 8};
    for (int M : Ms) {
        int64_t P = 1;
        while (P * M < n) P <<= 1;
        if (P > 64) continue;
        TileShape sh;
        sh.kernel = 3;
        sh.M = M;
        sh.P = (int)P;
        sh.contig = false;
        const int64_t maxt = dtype == TDMA_F64 && M == 32 ? 512 : 1024;
        int S_log2 = dtype == TDMA_F64 ? 4 : 5;
        while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > maxt) --S_log2;
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
        sh.S_log2 = S_log2;
        if (!shift_supported(dtype, sh)) continue;
        // FP64, 32 rows per lane, 16 or 32 partitions covering n: the kernel
        // that recomputes its pivots fits 32 systems (256-byte rows)
        if (dtype == TDMA_F64 && M == 32 && (P == 16 || P == 32) && P * M == n) {
            TileShape w = sh;
            w.kernel = 7;
            w.S_log2 = 5;
            while (w.S_log2 > 0 && ((int64_t)1 << (w.S_log2 - 1)) >= nsys) --w.S_log2;
            if (w.S_log2 > sh.S_log2 && shift_supported(dtype, w)) sh = w;
        }
        *out = sh;
        return true;
    }
    return false;
}

// Per-row coefficients on strided layouts: the walking kernel with 128-byte
// tile rows (16 FP64 systems; 16 FP32 systems, 64 bytes).  32 rows per lane
// (512 lanes) where n is at least 512, else 16; shapes whose partitions cover
// n exactly (no padding rows) first.  On the 1024^3 per-row z-lines (FP64):
// 32 rows per lane 10.2 ms, 16 rows 12.6 ms, 16 rows with 64-byte tile rows
// 20.4 ms.
static bool default_perrow_shape(int dtype, int64_t n, int64_t nsys, TileShape *out) {
    const int Ms[] = {32, 16};
    TileShape best;
    bool found = false, best_full = false;
    for (int M : Ms) {
        if (M == 32 && n < 512) continue;
        int64_t P = 2;
        while (P * M < n) P <<= 1;
        if (P > 64) continue;
        TileShape sh;
        sh.kernel = 5;
        sh.M = M;
        sh.P = (int)P;
        sh.contig = false;
        const int64_t maxt = M == 32 ? 512 : 1024;
        int S_log2 = 4;
        while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > maxt) --S_log2;
        while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
        sh.S_log2 = S_log2;
        if (!perrow_supported(dtype, sh)) continue;
        const bool full = P * M == n;
        if (!found || (full && !best_full)) {
            best = sh;
            best_full = full;
            found = true;
        }
    }
    if (found) *out = best;
    return found;
}

// Ragged layout: systems are bucketed by the power-of-two partition count
// they need; one launch per non-empty bucket (contiguous rows, LDS-staged).
// build_ragged_plan allocates the plan's device tables and uploads them
// synchronously; the caller owns them (free_ragged_plan).
// Bucket of a ragged system of len rows: M rows per lane (16 in FP64, up to
// 8,192 rows; 32 and 16 in FP32 at 6,144 rows), P the power of two that
// covers len / M.  With the four per-row arrays loaded at once and staged
// without bank conflicts, 16 rows per lane measured faster than 8 on the
// longest systems (6,144 rows: 118 against 143 us for 1,245 systems).
static void ragged_bucket(int dtype, int64_t len, int *M_out, int *P_out) {
    const int M = dtype == TDMA_F64 ? 16 : (len <= 6144 ? 32 : 16);
    const int64_t P = (len + M - 1) / M;
    int64_t Pb = 1;
    while (Pb < P) Pb <<= 1;
    *M_out = M;
    *P_out = (int)std::min<int64_t>(Pb, 1 << 30);
}

// min_block, the smallest block of the per-row tile list (lanes): on the
// 10,000 systems of 32..8192 rows (FP64) alone, blocks of 512 lanes
// throughout 248 us, 256 and 512 227 us, 128, 256 and 512 242 us (each block
// size is a launch of its own); beside the 768x512x1536 sweeps in a graph
// the 256-lane blocks take CUs from the sweeps (graph 6.79 -> 6.86 ms), so
// graphs build their plans with 512-lane blocks only.
int build_ragged_plan(const tdma_layout *L, int dtype, RaggedPlan *out, int min_block) {
    const int64_t nsys = L->nsys0;
    std::map<std::pair<int, int>, std::vector<int32_t>> buckets;   // (M, P) -> systems
    for (int64_t k = 0; k < nsys; ++k) {
        const int64_t len = L->offsets[k + 1] - L->offsets[k];
        int M, P;
        ragged_bucket(dtype, len, &M, &P);
        buckets[{M, P}].push_back((int32_t)k);
    }
    for (auto &kv : buckets)
        if (kv.first.second > fused_max_threads(dtype, kv.first.first))
            return fail(TDMA_EUNSUPPORTED, "a ragged system needs %d partitions of %d rows (max %d)",
                        kv.first.second, kv.first.first, fused_max_threads(dtype, kv.first.first));
    RaggedPlan rp;
    rp.nsys = nsys;
    rp.dtype = dtype;
    rp.offsets.assign(L->offsets, L->offsets + nsys + 1);
    std::vector<int32_t> all;
    for (auto &kv : buckets) {
        const int M = kv.first.first, P = kv.first.second;
        RaggedBucket b;
        b.shape.M = M;
        b.shape.P = P;
        b.shape.contig = true;
        int S_log2 = ilog2_floor(std::max(1, 256 / P));
        while (S_log2 > 0 && (P << S_log2) > fused_max_threads(dtype, M)) --S_log2;
        b.shape.S_log2 = S_log2;
        b.first = (int64_t)all.size();
        b.count = (int64_t)kv.second.size();
        all.insert(all.end(), kv.second.begin(), kv.second.end());
        rp.buckets.push_back(b);
    }
    // the tile-list form: per rows-per-lane class, tiles of every bucket
    // (longest systems first) whose S*P lanes fill a block of
    // max(min_block, P) lanes: smaller blocks let two run on a CU at once,
    // one block's loads beside the other's arithmetic (one launch per block
    // size)
    std::vector<RaggedTile> tiles;
    auto block_of = [&](int M, int P) {
        const int maxt = fused_max_threads(dtype, M);
        return std::min(maxt, std::max(min_block > 0 ? min_block : maxt, P));
    };
    std::vector<std::pair<int, int>> classes;   // (M, block lanes), largest blocks first
    for (const RaggedBucket &b : rp.buckets) {
        const std::pair<int, int> c{b.shape.M, block_of(b.shape.M, b.shape.P)};
        if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
    }
    std::sort(classes.begin(), classes.end(),
              [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                  return x.first != y.first ? x.first < y.first : x.second > y.second;
              });
    bool groups_ok = true;
    for (const auto &cl : classes) {
        const int M = cl.first;
        if (!fused_tiles_supported(dtype, M)) { groups_ok = false; break; }
        RaggedGroup g;
        g.M = M;
        g.threads = cl.second;
        g.first_tile = (int64_t)tiles.size();
        std::vector<const RaggedBucket *> bs;
        for (const RaggedBucket &b : rp.buckets)
            if (b.shape.M == M && block_of(M, b.shape.P) == cl.second) bs.push_back(&b);
        if (bs.empty()) continue;
        std::sort(bs.begin(), bs.end(),
                  [](const RaggedBucket *x, const RaggedBucket *y) { return x->shape.P > y->shape.P; });
        for (const RaggedBucket *b : bs) {
            const int P = b->shape.P;
            if (P > g.threads) { groups_ok = false; break; }
            const int S = g.threads / P;
            TileShape sh;
            sh.M = M;
            sh.P = P;
            sh.S_log2 = ilog2_floor(S);
            sh.contig = true;
            g.lds = std::max(g.lds, fused_lds_bytes(dtype, sh));
            for (int64_t k = 0; k < b->count; k += S) {
                RaggedTile t;
                t.first = (int32_t)(b->first + k);
                t.count = (int32_t)std::min<int64_t>(S, b->count - k);
                t.P_log2 = ilog2_floor(P);
                t.S_log2 = sh.S_log2;
                tiles.push_back(t);
            }
        }
        g.ntiles = (int64_t)tiles.size() - g.first_tile;
        if (g.lds > 160 * 1024) groups_ok = false;
        if (!groups_ok) break;
        rp.groups.push_back(g);
    }
    if (!groups_ok || tiles.size() > (size_t)INT32_MAX) {
        rp.groups.clear();
        tiles.clear();
    }
    hipError_t e = hipMalloc(&rp.d_offsets, (nsys + 1) * sizeof(int64_t));
    if (e != hipSuccess) return fail(TDMA_ENOMEM, "ragged offsets");
    e = hipMalloc(&rp.d_list, std::max<size_t>(1, all.size()) * sizeof(int32_t));
    if (e != hipSuccess) { (void)hipFree(rp.d_offsets); return fail(TDMA_ENOMEM, "ragged list"); }
    if (!tiles.empty()) {
        e = hipMalloc(&rp.d_tiles, tiles.size() * sizeof(RaggedTile));
        if (e != hipSuccess) {
            rp.d_tiles = nullptr;
            free_ragged_plan(&rp);
            return fail(TDMA_ENOMEM, "ragged tiles");
        }
    }
    e = hipMemcpy(rp.d_offsets, L->offsets, (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !all.empty())
        e = hipMemcpy(rp.d_list, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(rp.d_tiles, tiles.data(), tiles.size() * sizeof(RaggedTile), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_ragged_plan(&rp);
        return hip_fail(e, "upload ragged plan");
    }
    *out = rp;
    return TDMA_OK;
}

void free_ragged_plan(RaggedPlan *rp) {
    if (rp->d_offsets) (void)hipFree(rp->d_offsets);
    if (rp->d_list) (void)hipFree(rp->d_list);
    if (rp->d_tiles) (void)hipFree(rp->d_tiles);
    rp->d_tiles = nullptr;
    rp->d_offsets = nullptr;
    rp->d_list = nullptr;
}

// Plans of recently seen ragged layouts, keyed by a hash of the offsets and
// confirmed by comparing the offsets and dtype in full.
int plan_ragged(DeviceCtx *ctx, const tdma_layout *L, int dtype, const RaggedPlan **out) {
    const int64_t nsys = L->nsys0;
    uint64_t h = 1469598103934665603ull;
    for (int64_t k = 0; k <= nsys; ++k) {
        h ^= (uint64_t)L->offsets[k];
        h *= 1099511628211ull;
    }
    h ^= (uint64_t)dtype * 0x9E3779B97F4A7C15ull;
    auto it = ctx->ragged_cache.find(h);
    if (it != ctx->ragged_cache.end() && it->second.nsys == nsys && it->second.dtype == dtype &&
        std::equal(it->second.offsets.begin(), it->second.offsets.end(), L->offsets)) {
        *out = &it->second;
        return TDMA_OK;
    }
    RaggedPlan rp;
    int rc = build_ragged_plan(L, dtype, &rp);
    if (rc != TDMA_OK) return rc;
    if (ctx->ragged_cache.size() >= 8 || it != ctx->ragged_cache.end()) {
        // full (or a hash collision): drop the cached plans (the stream
        // order keeps launches already issued from them valid: their device
        // tables are freed only after a device synchronisation)
        (void)hipDeviceSynchronize();
        for (auto &kv : ctx->ragged_cache) free_ragged_plan(&kv.second);
        ctx->ragged_cache.clear();
    }
    auto res = ctx->ragged_cache.emplace(h, std::move(rp));
    *out = &res.first->second;
    return TDMA_OK;
}

SysMap make_map(const tdma_layout *L) {
    SysMap m;
    m.n = L->n;
    m.nsys = L->nsys0 * L->nsys1;
    m.nsys0 = std::max<int64_t>(1, L->nsys0);
    m.row_stride = L->row_stride;
    m.sys_stride0 = L->sys_stride0;
    m.sys_stride1 = L->sys_stride1;
    m.offsets = nullptr;
    m.sys_list = nullptr;
    m.count = nullptr;
    return m;
}

Coef make_coef(const tdma_coeffs *C) {
    Coef c;
    c.mode = C->mode;
    c.a = C->a;
    c.b = C->b;
    c.c = C->c;
    c.shift = C->b_shift;
    return c;
}

// Per-row coefficients without a shift: one launch per rows-per-lane class
// of the plan's tile list.  Otherwise one launch per bucket.
int launch_ragged(const RaggedPlan &rp, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                  const void *d, void *x, int *err, hipStream_t st, const hipStream_t *aux,
                  int naux, const hipEvent_t *ev) {
    const Coef coef = make_coef(C);
    if (C->mode == TDMA_COEF_LIKE_D && C->b_shift == nullptr && !rp.groups.empty()) {
        for (const RaggedGroup &g : rp.groups) {
            SysMap m = make_map(L);
            m.offsets = rp.d_offsets;
            m.sys_list = rp.d_list;
            const hipError_t e = launch_fused_tiles(dtype, g.M, m, coef, d, x, rp.d_tiles + g.first_tile,
                                                    g.ntiles, g.threads, g.lds, err, st);
            if (e != hipSuccess) return hip_fail(e, "fused launch (ragged tiles)");
        }
        return TDMA_OK;
    }
    const int nb = (int)rp.buckets.size();
    const int nuse = std::max(0, std::min(naux, nb - 1));
    hipError_t e = hipSuccess;
    if (nuse > 0) {
        e = hipEventRecord(ev[0], st);
        for (int i = 0; i < nuse && e == hipSuccess; ++i) e = hipStreamWaitEvent(aux[i], ev[0], 0);
        if (e != hipSuccess) return hip_fail(e, "ragged fork");
    }
    for (int k = 0; k < nb; ++k) {
        const RaggedBucket &b = rp.buckets[k];
        const int lane = k % (nuse + 1);
        SysMap m = make_map(L);
        m.n = (int64_t)b.shape.P * b.shape.M;
        m.nsys = b.count;
        m.offsets = rp.d_offsets;
        m.sys_list = rp.d_list + b.first;
        e = launch_fused(dtype, m, coef, b.shape, d, x, err, lane == 0 ? st : aux[lane - 1]);
        if (e != hipSuccess) return hip_fail(e, "fused launch (ragged)");
    }
    for (int i = 0; i < nuse && e == hipSuccess; ++i) {
        e = hipEventRecord(ev[1 + i], aux[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[1 + i], 0);
    }
    if (e != hipSuccess) return hip_fail(e, "ragged join");
    return TDMA_OK;
}

// Whether a tile shape can run a uniform layout with these coefficients.
static bool shape_fits(int dtype, const tdma_layout *L, bool shared_op, const TileShape &sh,
                       bool shifted_op, bool perrow_op) {
    if ((int64_t)sh.P * sh.M < L->n) return false;
    if (sh.kernel == 3 || sh.kernel == 4 || sh.kernel == 7) {
        if (!shifted_op || !shift_supported(dtype, sh)) return false;
        if (sh.kernel == 7 && (int64_t)sh.P * sh.M != L->n) return false;
        const SysMap m = make_map(L);
        return shift_layout_ok(m, sh);
    }
    if (sh.kernel == 5) return perrow_op && perrow_supported(dtype, sh) && perrow_layout_ok(make_map(L), sh);
    if (sh.kernel == 1 || sh.kernel == 2) return shared_op && shared_supported(dtype, sh);
    if (sh.kernel == 6) return shared_op && shared_supported(dtype, sh) && shared_roll_ok(make_map(L), sh);
    if (sh.kernel != 0 || !fused_supported(dtype, sh)) return false;
    return !(sh.contig && fused_lds_bytes(dtype, sh) > 160 * 1024);
}

// Tile shape of a uniform layout: the forced shape, else the autotune cache
// (an entry that no longer fits, e.g. from an edited cache file, is
// ignored), else the built-in rules (shared-operator kernel first where it
// applies).
int plan_uniform(DeviceCtx *ctx, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                 const TileShape *force, TileShape *out) {
    const int64_t nsys = L->nsys0 * L->nsys1;
    TileShape sh;
    const bool contig = L->row_stride == 1;
    const bool shared_op = C->mode == TDMA_COEF_SHARED && C->b_shift == nullptr;
    const bool shifted_op = C->mode == TDMA_COEF_SHARED && C->b_shift != nullptr;
    const bool perrow_op = C->mode == TDMA_COEF_LIKE_D && C->b_shift == nullptr;
    if (force) {
        sh = *force;
        if ((int64_t)sh.P * sh.M < L->n)
            return fail(TDMA_EINVAL, "tile shape M=%d P=%d S=%d does not cover n=%lld", sh.M, sh.P,
                        1 << sh.S_log2, (long long)L->n);
        if ((sh.kernel == 1 || sh.kernel == 2 || sh.kernel == 6) && !shared_op)
            return fail(TDMA_EINVAL, "the shared-operator kernel needs shared coefficients without "
                        "a shift (M=%d P=%d S=%d)", sh.M, sh.P, 1 << sh.S_log2);
        if ((sh.kernel == 3 || sh.kernel == 4 || sh.kernel == 7) && !shifted_op)
            return fail(TDMA_EINVAL, "the shifted-operator kernel needs shared coefficients with "
                        "a shift (M=%d P=%d S=%d)", sh.M, sh.P, 1 << sh.S_log2);
        if (sh.kernel == 5 && !perrow_op)
            return fail(TDMA_EINVAL, "the per-row kernel needs per-row coefficients without a "
                        "shift (M=%d P=%d S=%d)", sh.M, sh.P, 1 << sh.S_log2);
        if (!shape_fits(dtype, L, shared_op, sh, shifted_op, perrow_op))
            return fail(TDMA_EINVAL, "unsupported tile shape M=%d P=%d S=%d (kernel %d)", sh.M, sh.P,
                        1 << sh.S_log2, sh.kernel);
    } else if (!(lookup_tuned(ctx->dev, L, C, dtype, &sh) && sh.contig == contig &&
                 shape_fits(dtype, L, shared_op, sh, shifted_op, perrow_op))) {
        TileShape ssh;
        if (shifted_op && !contig && default_shift_shape(dtype, L->n, nsys, &ssh) &&
            shift_layout_ok(make_map(L), ssh))
            sh = ssh;
        else if (perrow_op && !contig && default_perrow_shape(dtype, L->n, nsys, &ssh) &&
                 perrow_layout_ok(make_map(L), ssh))
            sh = ssh;
        else if (shared_op && default_shared_shape(dtype, L->n, nsys, contig, &sh, true)) {
            if (sh.kernel == 6 && !shared_roll_ok(make_map(L), sh))
                default_shared_shape(dtype, L->n, nsys, contig, &sh, false);
        } else if (!default_shape(dtype, L->n, nsys, contig, &sh))
            return fail(TDMA_EUNSUPPORTED, "n = %lld is too long for the fused path (use "
                        "tdma_solve_partitioned)", (long long)L->n);
    }
    *out = sh;
    return TDMA_OK;
}

int launch_uniform(const TileShape &sh, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                   const void *d, void *x, int *err, hipStream_t st) {
    const SysMap m = make_map(L);
    if (m.nsys == 0) return TDMA_OK;
    const Coef coef = make_coef(C);
    hipError_t e;
    if (sh.kernel == 3 || sh.kernel == 4 || sh.kernel == 7)
        e = launch_shift(dtype, m, coef, sh, d, x, err, st);
    else if (sh.kernel == 5)
        e = launch_perrow(dtype, m, coef, sh, d, x, err, st);
    else if (sh.kernel != 0)
        e = launch_shared(dtype, m, coef, sh, d, x, err, st);
    else
        e = launch_fused(dtype, m, coef, sh, d, x, err, st);
    if (e != hipSuccess) return hip_fail(e, "fused launch");
    return TDMA_OK;
}

int run_fused(DeviceCtx *ctx, const tdma_layout *L, const tdma_coeffs *C, int dtype, const void *d,
              void *x, hipStream_t st, const TileShape *force) {
    if (L->offsets) {
        // A ragged call builds (or finds in the library's cache) a plan whose
        // device tables it allocates and uploads synchronously, and a cache
        // entry can later be freed: neither may happen inside, or be recorded
        // by, a capture the caller started.  Graphs of ragged solves are made
        // by tdma_graph_create, which gives them tables of their own.
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const hipError_t ce = hipStreamIsCapturing(st, &cs);
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
        if (cs != hipStreamCaptureStatusNone)
            return fail(TDMA_EUNSUPPORTED, "a ragged layout cannot be solved on a stream that is being "
                        "captured (use tdma_graph_create)");
        const RaggedPlan *rp = nullptr;
        int rc = plan_ragged(ctx, L, dtype, &rp);
        if (rc != TDMA_OK) return rc;
        // buckets on the caller's stream and kRaggedAux library streams at once
        hipStream_t *aux = nullptr;
        hipEvent_t *ev = nullptr;
        rc = ctx->get_streams(kRaggedAux, &aux);
        if (rc == TDMA_OK) rc = ctx->get_events(kRaggedAux + 1, &ev);
        if (rc != TDMA_OK) return rc;
        return launch_ragged(*rp, L, C, dtype, d, x, ctx->d_err, st, aux, kRaggedAux, ev);
    }
    if (L->nsys0 * L->nsys1 == 0) return TDMA_OK;
    TileShape sh;
    int rc = plan_uniform(ctx, L, C, dtype, force, &sh);
    if (rc != TDMA_OK) return rc;
    return launch_uniform(sh, L, C, dtype, d, x, ctx->d_err, st);
}

}  // namespace tdma

using namespace tdma;

extern "C" {

const char *tdma_status_string(int status) {
    switch (status) {
        case TDMA_OK: return "TDMA_OK";
        case TDMA_EINVAL: return "TDMA_EINVAL (invalid argument)";
        case TDMA_ENOMEM: return "TDMA_ENOMEM (allocation failed)";
        case TDMA_EHIP: return "TDMA_EHIP (HIP runtime error)";
        case TDMA_ESINGULAR: return "TDMA_ESINGULAR (zero or non-finite pivot)";
        case TDMA_ENOCONV: return "TDMA_ENOCONV (refinement did not converge)";
        case TDMA_EUNSUPPORTED: return "TDMA_EUNSUPPORTED (unsupported combination)";
        default: return "unknown tdma status";
    }
}

const char *tdma_last_error(void) { return g_last_error.c_str(); }

int tdma_solve_batched(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                       const void *d, void *x, void *stream) {
    clear_error();
    int rc = validate(layout, coeffs, dtype, d, x);
    if (rc != TDMA_OK) return rc;
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return run_fused(ctx, layout, coeffs, dtype, d, x, (hipStream_t)stream, nullptr);
}

int tdma_solve_batched_tiled(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                             const void *d, void *x, const tdma_tile *tile, void *stream) {
    clear_error();
    int rc = validate(layout, coeffs, dtype, d, x);
    if (rc != TDMA_OK) return rc;
    if (!tile) return fail(TDMA_EINVAL, "tile is NULL");
    if (layout->offsets) return fail(TDMA_EINVAL, "explicit tiles need a uniform layout");
    const int S = tile->systems_per_tile;
    if (S < 1 || (S & (S - 1)) != 0) return fail(TDMA_EINVAL, "systems_per_tile must be a power of two");
    TileShape sh;
    sh.M = tile->rows_per_lane;
    sh.P = tile->partitions;
    sh.S_log2 = 0;
    while ((1 << sh.S_log2) < S) ++sh.S_log2;
    sh.contig = layout->row_stride == 1;
    sh.kernel = tile->kernel;
    if (sh.kernel < 0 || sh.kernel > 7) return fail(TDMA_EINVAL, "unknown kernel %d", sh.kernel);
    if (sh.kernel == 0 && !fused_supported(dtype, sh))
        return fail(TDMA_EINVAL, "unsupported tile M=%d S=%d P=%d", sh.M, S, sh.P);
    if ((sh.kernel == 3 || sh.kernel == 4 || sh.kernel == 7) && !shift_supported(dtype, sh))
        return fail(TDMA_EINVAL, "unsupported shifted-operator tile M=%d S=%d P=%d", sh.M, S, sh.P);
    if (sh.kernel == 5 && !perrow_supported(dtype, sh))
        return fail(TDMA_EINVAL, "unsupported per-row tile M=%d S=%d P=%d", sh.M, S, sh.P);
    if ((sh.kernel == 1 || sh.kernel == 2 || sh.kernel == 6) && !shared_supported(dtype, sh))
        return fail(TDMA_EINVAL, "unsupported shared-operator tile M=%d S=%d P=%d", sh.M, S, sh.P);
    if (sh.kernel == 7 && (int64_t)sh.M * sh.P != layout->n)
        return fail(TDMA_EINVAL, "kernel 7 needs partitions that cover n exactly (M=%d P=%d, n = %lld)",
                    sh.M, sh.P, (long long)layout->n);
    if (sh.kernel == 6 && !shared_roll_ok(make_map(layout), sh))
        return fail(TDMA_EINVAL, "kernel 6 needs strided rows and partitions that cover n exactly "
                    "(M=%d P=%d, n = %lld)", sh.M, sh.P, (long long)layout->n);
    if ((int64_t)sh.M * sh.P < layout->n) return fail(TDMA_EINVAL, "tile covers %lld rows < n = %lld",
                                                      (long long)sh.M * sh.P, (long long)layout->n);
    if (sh.kernel == 0 && sh.contig && fused_lds_bytes(dtype, sh) > 160 * 1024)
        return fail(TDMA_EINVAL, "tile needs %zu bytes of LDS", fused_lds_bytes(dtype, sh));
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return run_fused(ctx, layout, coeffs, dtype, d, x, (hipStream_t)stream, &sh);
}

int tdma_copy_streamed(const tdma_layout *layout, int dtype, const void *src, void *dst,
                       void *stream) {
    clear_error();
    if (src == dst && src) return fail(TDMA_EINVAL, "src and dst must differ");
    tdma_coeffs none{};   // validation only, never read
    none.a = none.b = none.c = src;
    none.mode = TDMA_COEF_SHARED;
    int rc = validate(layout, &none, dtype, src, dst);
    if (rc != TDMA_OK) return rc;
    if (layout->offsets) return fail(TDMA_EUNSUPPORTED, "the streamed copy takes uniform layouts");
    if (layout->row_stride == 1)
        return fail(TDMA_EUNSUPPORTED, "the streamed copy follows the strided solve (row_stride != 1)");
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) return TDMA_OK;
    TileShape sh;
    if (!default_shared_shape(dtype, layout->n, nsys, false, &sh, false))
        return fail(TDMA_EUNSUPPORTED, "n = %lld has no streaming shape", (long long)layout->n);
    const SysMap map = make_map(layout);
    if (!copy_streamed_supported(map, sh))
        return fail(TDMA_EUNSUPPORTED, "layout beyond the streaming walk's 32-bit indices");
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipError_t e = launch_copy_streamed(dtype, map, sh, src, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "streamed copy launch");
    return TDMA_OK;
}

int tdma_solve_pdd(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                   int rows_per_partition, const void *d, void *x, void *stream) {
    clear_error();
    int rc = validate(layout, coeffs, dtype, d, x);
    if (rc != TDMA_OK) return rc;
    if (layout->offsets) return fail(TDMA_EINVAL, "the PDD solve takes uniform layouts");
    const int m = rows_per_partition;
    TileShape sh;
    sh.kernel = 0;
    sh.M = m;
    sh.pdd = true;
    sh.contig = layout->row_stride == 1;
    sh.S_log2 = 0;
    sh.P = 1;
    if (!fused_supported(dtype, sh))
        return fail(TDMA_EINVAL, "rows_per_partition = %d (4, 8 or 16; 32 too in FP32)", m);
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) return TDMA_OK;
    const int64_t P = (layout->n + m - 1) / m;
    const int maxt = fused_max_threads(dtype, m);
    if (P > maxt)
        return fail(TDMA_EUNSUPPORTED, "n = %lld needs %lld partitions of %d rows (at most %d)",
                    (long long)layout->n, (long long)P, m, maxt);
    sh.P = (int)P;
    const int esz = dtype == TDMA_F64 ? 8 : 4;
    int S_log2 = sh.contig ? ilog2_floor(std::max<int64_t>(1, 256 / P)) : ilog2_floor(128 / esz);
    while (S_log2 > 0 && ((int64_t)1 << S_log2) * P > maxt) --S_log2;
    while (S_log2 > 0 && ((int64_t)1 << (S_log2 - 1)) >= nsys) --S_log2;
    sh.S_log2 = S_log2;
    while (sh.contig && sh.S_log2 > 0 && fused_lds_bytes(dtype, sh) > 96 * 1024) --sh.S_log2;
    if (sh.contig && fused_lds_bytes(dtype, sh) > 160 * 1024)
        return fail(TDMA_EUNSUPPORTED, "a tile of n = %lld contiguous rows exceeds the LDS",
                    (long long)layout->n);
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return launch_uniform(sh, layout, coeffs, dtype, d, x, ctx->d_err, (hipStream_t)stream);
}

int tdma_solve_multi(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype, int nrhs,
                     int64_t rhs_stride, const void *d, void *x, void *stream) {
    clear_error();
    int rc = validate(layout, coeffs, dtype, d, x);
    if (rc != TDMA_OK) return rc;
    if (layout->offsets) return fail(TDMA_EINVAL, "several right-hand sides need a uniform layout");
    if (coeffs->mode != TDMA_COEF_SHARED)
        return fail(TDMA_EUNSUPPORTED, "several right-hand sides share one operator "
                                       "(mode TDMA_COEF_SHARED)");
    if (nrhs < 1) return fail(TDMA_EINVAL, "nrhs = %d (< 1)", nrhs);
    if (rhs_stride < 0) return fail(TDMA_EINVAL, "negative rhs_stride");
    if (nrhs > 1 && rhs_stride == 0) return fail(TDMA_EINVAL, "rhs_stride is 0 with nrhs = %d", nrhs);
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) return TDMA_OK;
    const __int128 last = (__int128)(layout->n - 1) * layout->row_stride +
                          (__int128)(layout->nsys0 - 1) * layout->sys_stride0 +
                          (__int128)(layout->nsys1 - 1) * layout->sys_stride1 +
                          (__int128)(nrhs - 1) * rhs_stride;
    if (last >= ((__int128)1 << 62))
        return fail(TDMA_EINVAL, "the layout and its right-hand sides span more than 2^62 elements");
    MultiShape sh;
    if (!multi_shape(dtype, layout->n, nsys, &sh))
        return fail(TDMA_EUNSUPPORTED, "n = %lld is longer than the %d rows the multi-right-hand-side "
                    "kernel holds", (long long)layout->n, dtype == TDMA_F64 ? 1024 : 2048);
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    const auto even = [](int64_t v) { return (v & 1) == 0; };
    const bool vec = nrhs >= 2 && rhs_stride == 1 && even(layout->row_stride) &&
                     (layout->nsys0 == 1 || even(layout->sys_stride0)) &&
                     (layout->nsys1 == 1 || even(layout->sys_stride1)) &&
                     (uintptr_t)d % (2 * esz) == 0 && (uintptr_t)x % (2 * esz) == 0;
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipError_t e = launch_multi(dtype, make_map(layout), make_coef(coeffs), sh, nrhs,
                                      rhs_stride, vec, d, x, ctx->d_err, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "multi-right-hand-side launch");
    return TDMA_OK;
}

int tdma_check(void *stream) {
    clear_error();
    DeviceCtx *ctx = nullptr;
    int rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::lock_guard<std::mutex> lk(ctx->mu);
    int flag[4] = {0, 0, 0, 0};
    e = hipMemcpy(flag, ctx->d_err, sizeof flag, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read error flag");
    if (flag[0]) {
        e = hipMemset(ctx->d_err, 0, 4 * sizeof(int));
        if (e != hipSuccess) return hip_fail(e, "clear error flag");
        return fail(TDMA_ESINGULAR, "a kernel met a zero or non-finite pivot");
    }
    return TDMA_OK;
}

void tdma_shutdown(void) {
    std::lock_guard<std::mutex> g(g_mutex);
    g_ctx.clear();
    clear_tuned();
}

}  // extern "C"
