// Batching form: a list of solves recorded once into a hipGraph that
// tdma_graph_launch replays as one submission.
//
// Each item is planned exactly as tdma_solve_batched would plan it (tuned or
// built-in tile shape, the shared-operator kernel where it applies, one
// launch per length bucket of a ragged batch), and its launches are recorded
// into the graph:
//   - items that read another item's output, and the items they read, go on
//     the main branch in item order, so a graph edge (kernel boundary) orders
//     every item after the one it reads;
//   - independent items go on a second branch forked from the start and
//     joined at the end, so the GPU runs them beside the dependent chain and
//     they fill its launch tails.
// There is no device-side waiting between workgroups: ordering comes only
// from the graph's edges.  Ragged plans (offsets and bucketed system lists)
// are uploaded before capture into memory the graph owns.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include <mutex>

#include "api_internal.h"

struct tdma_graph {
    int dev = 0;
    int dtype = 0;
    std::vector<tdma::RaggedPlan> ragged;   // device tables owned by the graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace tdma {
namespace {

void destroy_graph(tdma_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (RaggedPlan &rp : g->ragged) free_ragged_plan(&rp);
    delete g;
}

// One item's launches, planned before capture.
struct ItemPlan {
    bool ragged = false;
    int ragged_index = -1;   // into tdma_graph::ragged
    TileShape shape;
    bool empty = false;
    bool side = false;       // independent: recorded on the second branch
};

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
    }
    DeviceCtx *ctx = nullptr;
    int rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    tdma_graph *g = new tdma_graph();
    g->dev = ctx->dev;
    g->dtype = dtype;

    // 1. plans (host validation of every item before anything is recorded)
    std::vector<bool> needed(nitems, false);
    for (int i = 0; i < nitems; ++i)
        if (items[i].after >= 0) needed[items[i].after] = true;
    std::vector<ItemPlan> plans(nitems);
    for (int i = 0; i < nitems && rc == TDMA_OK; ++i) {
        const tdma_work_item &it = items[i];
        ItemPlan &pl = plans[i];
        pl.side = it.after < 0 && !needed[i];
        if (it.layout.offsets) {
            pl.ragged = true;
            if (it.layout.nsys0 == 0) { pl.empty = true; continue; }
            RaggedPlan rp;
            rc = build_ragged_plan(&it.layout, dtype, &rp, 0);   // beside the chain: full blocks
            if (rc != TDMA_OK) break;
            pl.ragged_index = (int)g->ragged.size();
            g->ragged.push_back(rp);
        } else {
            if (it.layout.nsys0 * it.layout.nsys1 == 0) { pl.empty = true; continue; }
            rc = plan_uniform(ctx, &it.layout, &it.coeffs, dtype, nullptr, &pl.shape);
            if (rc != TDMA_OK) {
                const std::string why = tdma_last_error();
                rc = fail(rc, "item %d: %s", i, why.c_str());
            }
        }
    }
    if (rc != TDMA_OK) { destroy_graph(g); return rc; }
    bool any_side = false, any_main = false;
    for (const ItemPlan &pl : plans) {
        if (pl.empty) continue;
        (pl.side ? any_side : any_main) = true;
    }

    // 2. record: main branch on `cap`, independent items on `side`
    hipStream_t cap = nullptr, side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e != hipSuccess) rc = hip_fail(e, "graph streams");
    bool capturing = false;
    if (rc == TDMA_OK) {
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = hip_fail(e, "begin capture");
        else capturing = true;
    }
    if (rc == TDMA_OK && any_side && any_main) {
        e = hipEventRecord(fork, cap);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
        if (e != hipSuccess) rc = hip_fail(e, "fork");
    }
    for (int i = 0; i < nitems && rc == TDMA_OK; ++i) {
        const ItemPlan &pl = plans[i];
        if (pl.empty) continue;
        const tdma_work_item &it = items[i];
        hipStream_t st = pl.side && any_main ? side : cap;
        if (pl.ragged)
            rc = launch_ragged(g->ragged[pl.ragged_index], &it.layout, &it.coeffs, dtype, it.d, it.x,
                               ctx->d_err, st, nullptr, 0, nullptr);
        else
            rc = launch_uniform(pl.shape, &it.layout, &it.coeffs, dtype, it.d, it.x, ctx->d_err, st);
    }
    if (rc == TDMA_OK && any_side && any_main) {
        e = hipEventRecord(join, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(cap, join, 0);
        if (e != hipSuccess) rc = hip_fail(e, "join");
    }
    hipGraph_t graph = nullptr;
    if (capturing) {
        e = hipStreamEndCapture(cap, &graph);
        if (rc == TDMA_OK && e != hipSuccess) rc = hip_fail(e, "end capture");
    }
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
    if (cap) (void)hipStreamDestroy(cap);
    if (rc != TDMA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        destroy_graph(g);
        return rc;
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
