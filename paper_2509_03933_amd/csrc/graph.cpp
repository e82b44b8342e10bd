// Batching form host side: plan the work items into tiles and a dependency-
// ordered queue, then record [counter reset; persistent kernel] into a
// hipGraph that tdma_graph_launch replays.
#include <algorithm>
#include <cstring>
#include <vector>

#include "api_internal.h"
#include "persist.h"

struct tdma_graph {
    int dev = 0;
    int dtype = 0;
    void *dmem = nullptr;          // descriptors, segments, counters
    std::vector<void *> owned;     // device copies of ragged offsets and system lists
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace tdma {
namespace {

void destroy_graph(tdma_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (void *p : g->owned) (void)hipFree(p);
    if (g->dmem) (void)hipFree(g->dmem);
    delete g;
}

// Tile of the persistent kernel: M rows per lane, P a power of two covering
// n, S = 1024 / P systems.
bool persist_shape(int64_t n, int dtype, bool contig, int *S_log2, int *P) {
    const int M = persist_rows_per_lane();
    int p = 1;
    while ((int64_t)p * M < n) p <<= 1;
    if (p > kPersistThreads) return false;
    int s_log2 = 0;
    while ((p << (s_log2 + 1)) <= kPersistThreads) ++s_log2;
    TileShape sh;
    sh.M = M;
    sh.P = p;
    sh.S_log2 = s_log2;
    sh.contig = contig;
    if (!fused_supported(dtype, sh) || fused_lds_bytes(dtype, sh) > 160 * 1024) return false;
    *S_log2 = s_log2;
    *P = p;
    return true;
}

}  // namespace
}  // namespace tdma

using namespace tdma;

extern "C" int tdma_graph_create(const tdma_work_item *items, int nitems, int dtype, tdma_graph **out) {
    clear_error();
    if (!out) return fail(TDMA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!items || nitems < 1) return fail(TDMA_EINVAL, "no work items");
    if (dtype != TDMA_F64 && dtype != TDMA_F32) return fail(TDMA_EINVAL, "unknown dtype %d", dtype);
    for (int i = 0; i < nitems; ++i) {
        int rc = validate(&items[i].layout, &items[i].coeffs, dtype, items[i].d, items[i].x);
        if (rc != TDMA_OK) return rc;
        if (items[i].after >= i || items[i].after < -1)
            return fail(TDMA_EINVAL, "item %d: after = %d must name an earlier item", i, items[i].after);
        if (items[i].after >= 0 && items[items[i].after].layout.offsets)
            return fail(TDMA_EUNSUPPORTED, "item %d depends on a ragged item", i);
    }
    DeviceCtx *ctx = nullptr;
    int rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    tdma_graph *g = new tdma_graph();
    g->dev = ctx->dev;
    g->dtype = dtype;
    const int M = persist_rows_per_lane();

    // 1. descriptors (ragged items become one descriptor per length class)
    std::vector<WorkDesc> descs;
    std::vector<int> item_desc(nitems, -1);
    std::vector<bool> filler;          // independent of everything, nobody waits for it
    std::vector<bool> needed(nitems, false);
    for (int i = 0; i < nitems; ++i)
        if (items[i].after >= 0) needed[items[i].after] = true;
    size_t lds = 0;
    for (int i = 0; i < nitems && rc == TDMA_OK; ++i) {
        const tdma_work_item &it = items[i];
        const tdma_layout &L = it.layout;
        WorkDesc wd;
        std::memset(&wd, 0, sizeof wd);
        wd.map = make_map(&L);
        wd.coef = make_coef(&it.coeffs);
        wd.d = it.d;
        wd.x = it.x;
        wd.like_d = it.coeffs.mode == TDMA_COEF_LIKE_D;
        wd.shift = it.coeffs.b_shift != nullptr;
        wd.after = it.after >= 0 ? item_desc[it.after] : -1;
        const bool indep = it.after < 0 && !needed[i];
        if (!L.offsets) {
            if (wd.map.nsys == 0) continue;
            wd.contig = L.row_stride == 1;
            if (!persist_shape(L.n, dtype, wd.contig, &wd.S_log2, &wd.P)) {
                rc = fail(TDMA_EUNSUPPORTED, "item %d: n = %lld is too long for the batching form",
                          i, (long long)L.n);
                break;
            }
            wd.ntiles = (wd.map.nsys + (1 << wd.S_log2) - 1) >> wd.S_log2;
            item_desc[i] = (int)descs.size();
            descs.push_back(wd);
            filler.push_back(indep);
        } else {
            const int64_t nsys = L.nsys0;
            std::vector<std::vector<int32_t>> cls(11);
            for (int64_t k = 0; k < nsys; ++k) {
                const int64_t len = L.offsets[k + 1] - L.offsets[k];
                int c = 0;
                while (((int64_t)1 << c) * M < len) ++c;
                if (c > 10) { rc = fail(TDMA_EUNSUPPORTED, "item %d: a ragged system is too long", i); break; }
                cls[c].push_back((int32_t)k);
            }
            if (rc != TDMA_OK) break;
            int64_t *doff = nullptr;
            if (hipMalloc(&doff, (nsys + 1) * sizeof(int64_t)) != hipSuccess ||
                hipMemcpy(doff, L.offsets, (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
                rc = fail(TDMA_ENOMEM, "ragged offsets");
                break;
            }
            g->owned.push_back(doff);
            for (int c = 0; c <= 10 && rc == TDMA_OK; ++c) {
                if (cls[c].empty()) continue;
                int32_t *dl = nullptr;
                if (hipMalloc(&dl, cls[c].size() * sizeof(int32_t)) != hipSuccess ||
                    hipMemcpy(dl, cls[c].data(), cls[c].size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
                    rc = fail(TDMA_ENOMEM, "ragged system list");
                    break;
                }
                g->owned.push_back(dl);
                WorkDesc rd = wd;
                rd.contig = 1;
                rd.P = 1 << c;
                rd.S_log2 = 0;
                while ((rd.P << (rd.S_log2 + 1)) <= kPersistThreads) ++rd.S_log2;
                rd.map.n = (int64_t)rd.P * M;
                rd.map.nsys = (int64_t)cls[c].size();
                rd.map.offsets = doff;
                rd.map.sys_list = dl;
                rd.ntiles = (rd.map.nsys + (1 << rd.S_log2) - 1) >> rd.S_log2;
                TileShape sh;
                sh.M = M; sh.P = rd.P; sh.S_log2 = rd.S_log2; sh.contig = true;
                if (!fused_supported(dtype, sh) || fused_lds_bytes(dtype, sh) > 160 * 1024) {
                    rc = fail(TDMA_EUNSUPPORTED, "item %d: ragged tile does not fit", i);
                    break;
                }
                descs.push_back(rd);
                filler.push_back(true);
            }
        }
    }
    if (rc == TDMA_OK && (descs.empty() || descs.size() > (size_t)kMaxWorkDescs))
        rc = fail(descs.empty() ? TDMA_EINVAL : TDMA_EUNSUPPORTED, "%zu work descriptors (1..%d)",
                  descs.size(), kMaxWorkDescs);
    if (rc != TDMA_OK) { destroy_graph(g); return rc; }
    for (const WorkDesc &wd : descs) {
        TileShape sh;
        sh.M = M; sh.P = wd.P; sh.S_log2 = wd.S_log2; sh.contig = wd.contig != 0;
        lds = std::max(lds, fused_lds_bytes(dtype, sh));
    }

    // 2. occupancy: a grid every block of which can be resident
    int per_cu = 0;
    hipError_t e = persist_occupancy(dtype, lds, &per_cu);
    if (e != hipSuccess || per_cu < 1) {
        destroy_graph(g);
        return e != hipSuccess ? hip_fail(e, "occupancy") : fail(TDMA_EUNSUPPORTED, "persistent block does not fit a CU");
    }
    const int grid = per_cu * ctx->num_cus;

    // 3. queue order: dependent descriptors in order, fillers cut into chunks
    //    placed right after each descriptor that someone waits for
    std::vector<WorkSeg> segs;
    int64_t pos = 0;
    std::vector<int64_t> filler_next(descs.size(), 0);
    auto push = [&](int di, int64_t begin, int64_t count) {
        if (count <= 0) return;
        segs.push_back(WorkSeg{di, begin, count, pos});
        pos += count;
    };
    auto push_fillers = [&](int64_t budget) {
        for (size_t di = 0; di < descs.size() && budget > 0; ++di) {
            if (!filler[di]) continue;
            const int64_t take = std::min(budget, descs[di].ntiles - filler_next[di]);
            push((int)di, filler_next[di], take);
            filler_next[di] += take;
            budget -= take;
        }
    };
    for (size_t di = 0; di < descs.size(); ++di) {
        if (filler[di]) continue;
        push((int)di, 0, descs[di].ntiles);
        bool waited_on = false;
        for (const WorkDesc &o : descs) waited_on |= o.after == (int)di;
        if (waited_on) push_fillers(2 * (int64_t)grid);
    }
    push_fillers(INT64_MAX);
    const int64_t total_tiles = pos;

    // 4. device tables
    const size_t desc_b = (descs.size() * sizeof(WorkDesc) + 255) & ~(size_t)255;
    const size_t seg_b = (segs.size() * sizeof(WorkSeg) + 255) & ~(size_t)255;
    e = hipMalloc(&g->dmem, desc_b + seg_b + sizeof(WorkCounters));
    if (e != hipSuccess) { destroy_graph(g); return fail(TDMA_ENOMEM, "graph tables"); }
    WorkDesc *d_desc = (WorkDesc *)g->dmem;
    WorkSeg *d_seg = (WorkSeg *)((char *)g->dmem + desc_b);
    WorkCounters *d_ctr = (WorkCounters *)((char *)g->dmem + desc_b + seg_b);
    e = hipMemcpy(d_desc, descs.data(), descs.size() * sizeof(WorkDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_seg, segs.data(), segs.size() * sizeof(WorkSeg), hipMemcpyHostToDevice);
    if (e != hipSuccess) { destroy_graph(g); return hip_fail(e, "graph tables upload"); }

    // 5. record [reset; persistent kernel] into a graph
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) { destroy_graph(g); return hip_fail(e, "capture stream"); }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_persist_reset(d_ctr, (int)descs.size(), cap);
    if (e == hipSuccess)
        e = launch_persist(dtype, grid, lds, d_desc, d_seg, (int)segs.size(), total_tiles, d_ctr,
                           ctx->d_err, cap);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = e2;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        destroy_graph(g);
        return hip_fail(e, "graph capture");
    }
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { destroy_graph(g); return hip_fail(e, "graph instantiate"); }
    *out = g;
    return TDMA_OK;
}

extern "C" int tdma_graph_launch(tdma_graph *graph, void *stream) {
    clear_error();
    if (!graph || !graph->exec) return fail(TDMA_EINVAL, "graph is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != graph->dev) return fail(TDMA_EINVAL, "graph was created on device %d", graph->dev);
    e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return TDMA_OK;
}

extern "C" void tdma_graph_destroy(tdma_graph *graph) { destroy_graph(graph); }
