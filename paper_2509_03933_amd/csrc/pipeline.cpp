// tdma_solve_partitioned: batch formation and the stream pipeline.
//
// Systems are cut into batches of `batch` systems (the paper's batch_z, with
// a smaller remainder batch, Sec. 4.2.1).  Each batch runs Stage A, B and C
// (partitioned.hip).  Schedule 0 follows Algorithm 2: three consecutive
// batches are in flight -- at step n, Stage A of batch n, Stage B of batch
// n-1 and Stage C of batch n-2 are issued; A and C go to the "scalable" stream
// role, B to the "non-scalable" role, and hipEvents replace the host
// synchronisations, so no host wait happens inside the loop.  Out-of-range
// batch indices are skipped.  Workspaces (factors, reduced rows, interface
// solutions) are triple-buffered by batch index mod 3.  Schedule 1 gives each
// batch all three stages on stream (batch mod nstreams).
#include <algorithm>
#include <vector>

#include <mutex>

#include "api_internal.h"
#include "partitioned.h"

namespace tdma {

struct SlotBufs {
    void *ws_d, *ws_a, *ws_c;
    double *red, *X, *scratch;
};

int pipeline_solve(DeviceCtx *ctx, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                   const void *d, void *x, int P, int64_t batch, int nstreams, int schedule,
                   hipStream_t caller) {
    const SysMap map = make_map(L);
    const Coef coef = make_coef(C);
    const int64_t nsys = map.nsys;
    if (nsys == 0) return TDMA_OK;
    const int64_t n = L->n;
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    batch = std::max<int64_t>(1, std::min(batch, nsys));
    const int64_t nbatches = (nsys + batch - 1) / batch;
    const bool shared_factors = C->mode == TDMA_COEF_SHARED && C->b_shift == nullptr;
    int nslots = schedule == 0 ? 3 : nstreams;
    nslots = (int)std::max<int64_t>(1, std::min<int64_t>(nslots, nbatches));

    // per-slot workspace
    const size_t fac = shared_factors ? (size_t)n : (size_t)n * batch;
    const size_t fac_bytes = (fac * esz + 255) & ~(size_t)255;
    const size_t dh_bytes = ((size_t)n * batch * esz + 255) & ~(size_t)255;
    const size_t red_bytes = ((size_t)6 * P * batch * 8 + 255) & ~(size_t)255;
    const size_t x_bytes = ((size_t)2 * P * batch * 8 + 255) & ~(size_t)255;
    const size_t slot_bytes = dh_bytes + 2 * fac_bytes + red_bytes + 2 * x_bytes;
    void *ws = nullptr;
    int rc = ctx->workspace(1, slot_bytes * nslots, &ws);
    if (rc != TDMA_OK) return rc;
    std::vector<SlotBufs> slots(nslots);
    for (int i = 0; i < nslots; ++i) {
        char *b = (char *)ws + slot_bytes * i;
        slots[i].ws_d = b;
        b += dh_bytes;
        slots[i].ws_a = b;
        slots[i].ws_c = b + fac_bytes;
        slots[i].red = (double *)(b + 2 * fac_bytes);
        slots[i].X = (double *)(b + 2 * fac_bytes + red_bytes);
        slots[i].scratch = (double *)(b + 2 * fac_bytes + red_bytes + x_bytes);
    }

    hipStream_t *streams = nullptr;
    rc = ctx->get_streams(nstreams, &streams);
    if (rc != TDMA_OK) return rc;
    hipEvent_t *ev = nullptr;
    // events: [0] fork, [1 .. nstreams] joins, then evA/evB/evC per slot
    const int ev_base = 1 + nstreams;
    rc = ctx->get_events(ev_base + 3 * nslots, &ev);
    if (rc != TDMA_OK) return rc;
    hipEvent_t *evA = ev + ev_base, *evB = evA + nslots, *evC = evB + nslots;

    hipError_t e = hipEventRecord(ev[0], caller);
    for (int i = 0; i < nstreams && e == hipSuccess; ++i) e = hipStreamWaitEvent(streams[i], ev[0], 0);
    if (e != hipSuccess) return hip_fail(e, "pipeline fork");

    const int nAC = nstreams == 1 ? 1 : nstreams / 2;
    const int nB = nstreams == 1 ? 1 : nstreams - nAC;
    auto ac_stream = [&](int64_t b) { return streams[b % nAC]; };
    auto b_stream = [&](int64_t b) { return nstreams == 1 ? streams[0] : streams[nAC + b % nB]; };
    auto nb_of = [&](int64_t b) { return std::min(batch, nsys - b * batch); };

    auto stage_a = [&](int64_t b, hipStream_t s) {
        const SlotBufs &sb = slots[b % nslots];
        return launch_stage_a(dtype, map, coef, d, sb.ws_d, sb.ws_a, sb.ws_c, sb.red, b * batch,
                              nb_of(b), P, shared_factors, ctx->d_err, s);
    };
    auto stage_b = [&](int64_t b, hipStream_t s) {
        const SlotBufs &sb = slots[b % nslots];
        return launch_stage_b(sb.red, sb.X, sb.scratch, nb_of(b), P, ctx->d_err, s);
    };
    auto stage_c = [&](int64_t b, hipStream_t s) {
        const SlotBufs &sb = slots[b % nslots];
        return launch_stage_c(dtype, map, x, sb.ws_d, sb.ws_a, sb.ws_c, sb.X, b * batch, nb_of(b), P,
                              shared_factors, s);
    };

    if (schedule == 0) {
        for (int64_t it = 0; it < nbatches + 2 && e == hipSuccess; ++it) {
            if (it < nbatches) {
                const int64_t b = it;
                const int sl = (int)(b % nslots);
                hipStream_t s = ac_stream(b);
                if (b >= nslots) e = hipStreamWaitEvent(s, evC[sl], 0);   // slot reuse
                if (e == hipSuccess) e = stage_a(b, s);
                if (e == hipSuccess) e = hipEventRecord(evA[sl], s);
            }
            if (it >= 1 && it <= nbatches && e == hipSuccess) {
                const int64_t b = it - 1;
                const int sl = (int)(b % nslots);
                hipStream_t s = b_stream(b);
                e = hipStreamWaitEvent(s, evA[sl], 0);
                if (e == hipSuccess) e = stage_b(b, s);
                if (e == hipSuccess) e = hipEventRecord(evB[sl], s);
            }
            if (it >= 2 && e == hipSuccess) {
                const int64_t b = it - 2;
                const int sl = (int)(b % nslots);
                hipStream_t s = ac_stream(b);
                e = hipStreamWaitEvent(s, evB[sl], 0);
                if (e == hipSuccess) e = stage_c(b, s);
                if (e == hipSuccess) e = hipEventRecord(evC[sl], s);
            }
        }
    } else {
        for (int64_t b = 0; b < nbatches && e == hipSuccess; ++b) {
            hipStream_t s = streams[b % nstreams];
            e = stage_a(b, s);
            if (e == hipSuccess) e = stage_b(b, s);
            if (e == hipSuccess) e = stage_c(b, s);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "pipeline launch");
    for (int i = 0; i < nstreams && e == hipSuccess; ++i) {
        e = hipEventRecord(ev[1 + i], streams[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(caller, ev[1 + i], 0);
    }
    if (e != hipSuccess) return hip_fail(e, "pipeline join");
    return TDMA_OK;
}

}  // namespace tdma

using namespace tdma;

extern "C" int tdma_solve_partitioned(const tdma_layout *layout, const tdma_coeffs *coeffs,
                                      int dtype, const void *d, void *x, const tdma_part_opts *opts,
                                      void *stream) {
    clear_error();
    int rc = validate(layout, coeffs, dtype, d, x);
    if (rc != TDMA_OK) return rc;
    if (layout->offsets) return fail(TDMA_EUNSUPPORTED, "the partitioned path takes uniform layouts");
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) return TDMA_OK;
    int P = opts ? opts->partitions : 0;
    int64_t batch = opts && opts->batch ? opts->batch : 0;
    int nstreams = opts && opts->nstreams ? opts->nstreams : 0;
    const int sched_opt = opts ? opts->schedule : 0;
    if (P < 0) return fail(TDMA_EINVAL, "partitions = %d (< 0)", P);
    if (P > 0 && layout->n / P < 2)
        return fail(TDMA_EINVAL, "n = %lld gives partitions of < 2 rows (P = %d)",
                    (long long)layout->n, P);
    if (P > 4096) return fail(TDMA_EINVAL, "partitions = %d (> 4096)", P);
    if (nstreams < 0 || nstreams > 8) return fail(TDMA_EINVAL, "nstreams = %d (1..8)", nstreams);
    if (sched_opt < 0 || sched_opt > 2) return fail(TDMA_EINVAL, "schedule = %d (0, 1 or 2)", sched_opt);
    if (batch < 0) return fail(TDMA_EINVAL, "batch = %lld (< 0)", (long long)batch);
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    // unset fields: the autotuned values for this shape if cached (with P
    // unset, the tuner's P too), else the measured defaults (P = 8, batches
    // of 32,768 systems, 4 streams, round robin)
    int64_t t_batch = 32768;
    int t_streams = 4, t_sched = 1;
    int tP = P;
    if (lookup_tuned_batch(ctx->dev, layout, coeffs, dtype, &tP, &t_batch, &t_streams, &t_sched))
        P = tP;
    if (P == 0) {
        P = 8;
        tP = P;
        (void)lookup_tuned_batch(ctx->dev, layout, coeffs, dtype, &tP, &t_batch, &t_streams, &t_sched);
    }
    if (layout->n / P < 2)
        return fail(TDMA_EINVAL, "n = %lld gives partitions of < 2 rows (P = %d)",
                    (long long)layout->n, P);
    if (batch == 0) batch = t_batch;
    if (nstreams == 0) nstreams = t_streams;
    // the pipeline's own numbering: 0 = stage roles, 1 = round robin
    const int schedule = sched_opt == 0 ? t_sched : (sched_opt == 1 ? 1 : 0);
    return pipeline_solve(ctx, layout, coeffs, dtype, d, x, P, batch, nstreams, schedule,
                          (hipStream_t)stream);
}
