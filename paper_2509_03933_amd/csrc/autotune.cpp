// Autotuner: tile shapes of the fused path, batch size of the staged path.
//
// Fused path: every applicable tile shape (kernel variant, rows per lane M,
// systems per tile S, partitions P) is timed with hipEvents on the caller's
// buffers; the fastest is cached for this shape.
//
// Staged path (the paper's batch-size optimisation, Sec. 4.2.3: stage times
// measured on their own, total predicted by a model of the pipelined
// schedule): for each partition count P (2..32, n/P >= 2) and batch size s
// (powers of two from 2^12 to 2^18, clipped to the number of systems), the
// time of Stage A, B and C is measured for one batch alone and for K = 4
// batches at once on the pipeline's streams, each repetition on other
// batches (so no batch is served from the caches by the previous
// repetition).  The model is the schedule the pipeline runs by default,
// round robin over K streams (round_robin_model_ms): N_b = ceil(N/s)
// batches in rounds of K.  The paper's Algorithm 2 model (pipeline_model_ms:
// Stage B of batch k-1 beside A of batch k and C of batch k-2) is recorded
// too; on one GPU its stage roles leave the concurrency of the streams out,
// and with stage times of a batch alone it misranks the candidates.  The
// argmin is cached.  Mode 2 also runs the full pipeline for every candidate
// (brute force) and records both, so the model's choice can be checked
// against the measured best.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "api_internal.h"
#include "partitioned.h"

namespace tdma {

namespace {

struct Tuned {
    TileShape shape;
    bool has_shape = false;
    int64_t batch = 0;
    int nstreams = 4;
    int schedule = 0;
    int P = 0;
};

// streams of the staged pipeline the tuner tunes for (its default count)
constexpr int kTuneStreams = 4;

std::mutex g_tune_mutex;
std::map<std::string, Tuned> g_tuned;
bool g_cache_loaded = false;
std::string g_last_json = "{}";

std::string key_of(int dev, const tdma_layout *L, const tdma_coeffs *C, int dtype, const char *path,
                   int P) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s|dev%d|n%lld|s%lldx%lld|rs%lld|ss%lld,%lld|m%d|sh%d|dt%d|P%d", path,
             dev, (long long)L->n, (long long)L->nsys0, (long long)L->nsys1,
             (long long)L->row_stride, (long long)L->sys_stride0, (long long)L->sys_stride1, C->mode,
             C->b_shift ? 1 : 0, dtype, P);
    return buf;
}

// Cache file (TDMA_CACHE): one line per entry, whitespace-separated:
// "key has_shape kernel M S_log2 P contig batch nstreams schedule P"
void load_cache_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char *path = getenv("TDMA_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        Tuned t;
        int hs = 0, contig = 0;
        if (is >> key >> hs >> t.shape.kernel >> t.shape.M >> t.shape.S_log2 >> t.shape.P >> contig >>
            t.batch >> t.nstreams >> t.schedule >> t.P) {
            t.has_shape = hs != 0;
            t.shape.contig = contig != 0;
            g_tuned[key] = t;
        }
    }
}

void save_cache_locked() {
    const char *path = getenv("TDMA_CACHE");
    if (!path) return;
    std::ofstream f(path);
    for (auto &kv : g_tuned) {
        const Tuned &t = kv.second;
        f << kv.first << ' ' << (t.has_shape ? 1 : 0) << ' ' << t.shape.kernel << ' ' << t.shape.M
          << ' ' << t.shape.S_log2 << ' ' << t.shape.P << ' ' << (t.shape.contig ? 1 : 0) << ' '
          << t.batch << ' ' << t.nstreams << ' ' << t.schedule << ' ' << t.P << '\n';
    }
}

// time `fn` (which enqueues work on st): 2 warm-up runs, median of `reps`
template <typename F>
int time_median(hipStream_t st, int reps, F fn, float *ms_out) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(TDMA_EHIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(TDMA_EHIP, "hipEventCreate");
    }
    int rc = TDMA_OK;
    std::vector<float> v;
    for (int i = 0; i < reps + 2 && rc == TDMA_OK; ++i) {
        hipError_t e = hipEventRecord(e0, st);
        if (e == hipSuccess) rc = fn();
        if (rc == TDMA_OK && e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess && rc == TDMA_OK) rc = hip_fail(e, "autotune timing");
        if (i >= 2) v.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TDMA_OK) return rc;
    std::sort(v.begin(), v.end());
    *ms_out = v[v.size() / 2];
    return TDMA_OK;
}

std::vector<TileShape> fused_candidates(int dtype, const tdma_layout *L, const tdma_coeffs *C) {
    std::vector<TileShape> out;
    const int64_t n = L->n, nsys = L->nsys0 * L->nsys1;
    const bool contig = L->row_stride == 1;
    const bool shared_op = C->mode == TDMA_COEF_SHARED && C->b_shift == nullptr;
    if (shared_op) {
        for (int M : {8, 12, 16, 24, 32}) {
            int P = 1;
            while ((int64_t)P * M < n) P <<= 1;
            if (P > 64) continue;
            for (int S_log2 = 0; S_log2 <= 6; ++S_log2) {
                for (int kind : {1, 2, 6}) {
                    // the rolling form (6): strided rows, partitions covering n
                    if (kind == 6 && (contig || (int64_t)P * M != n)) continue;
                    TileShape sh;
                    sh.kernel = kind; sh.M = M; sh.P = P; sh.S_log2 = S_log2; sh.contig = contig;
                    if ((1 << S_log2) * P < 64 && (int64_t)(1 << S_log2) < nsys) continue;
                    if (shared_supported(dtype, sh) && (kind != 6 || shared_roll_ok(make_map(L), sh)))
                        out.push_back(sh);
                }
            }
        }
    }
    // the walking kernels of strided layouts: shifted shared operator
    // (kernels 3, 4) and per-row coefficients (kernel 5)
    const bool shifted_op = C->mode == TDMA_COEF_SHARED && C->b_shift != nullptr;
    const bool perrow_op = C->mode == TDMA_COEF_LIKE_D && C->b_shift == nullptr;
    if (!contig && (shifted_op || perrow_op)) {
        const SysMap m = make_map(L);
        for (int M : {8, 16, 32}) {
            int P = 2;
            while ((int64_t)P * M < n) P <<= 1;
            if (P > 64) continue;
            for (int S_log2 = 2; S_log2 <= 5; ++S_log2) {
                for (int kind : {3, 4, 5, 7}) {
                    if ((kind == 5) != perrow_op) continue;
                    if (kind == 7 && (int64_t)P * M != n) continue;
                    TileShape sh;
                    sh.kernel = kind; sh.M = M; sh.P = P; sh.S_log2 = S_log2; sh.contig = false;
                    const bool ok = kind == 5 ? perrow_supported(dtype, sh) && perrow_layout_ok(m, sh)
                                              : shift_supported(dtype, sh) && shift_layout_ok(m, sh);
                    if (ok) out.push_back(sh);
                }
            }
        }
    }
    for (int M : {4, 8, 16, 32}) {
        const int64_t P0 = (n + M - 1) / M;
        int64_t P2 = 1;
        while (P2 < P0) P2 <<= 1;
        for (int64_t P : {P0, P2}) {
            if (P > 1024) continue;
            for (int S_log2 = 0; S_log2 <= 6; ++S_log2) {
                TileShape sh;
                sh.kernel = 0; sh.M = M; sh.P = (int)P; sh.S_log2 = S_log2; sh.contig = contig;
                if ((int64_t)(1 << S_log2) * P < 64 && (int64_t)(1 << S_log2) < nsys) continue;
                if (!fused_supported(dtype, sh)) continue;
                if (contig && fused_lds_bytes(dtype, sh) > 160 * 1024) continue;
                out.push_back(sh);
            }
            if (P2 == P0) break;
        }
    }
    return out;
}

}  // namespace

bool lookup_tuned(int dev, const tdma_layout *L, const tdma_coeffs *C, int dtype, TileShape *out) {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    load_cache_locked();
    auto it = g_tuned.find(key_of(dev, L, C, dtype, "fused", 0));
    if (it == g_tuned.end() || !it->second.has_shape) return false;
    *out = it->second.shape;
    return true;
}

bool lookup_tuned_batch(int dev, const tdma_layout *L, const tdma_coeffs *C, int dtype, int *P,
                        int64_t *batch, int *nstreams, int *schedule) {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    load_cache_locked();
    auto it = g_tuned.find(key_of(dev, L, C, dtype, "part", *P));
    if (it == g_tuned.end() || it->second.batch <= 0 || it->second.P < 1) return false;
    *P = it->second.P;
    *batch = it->second.batch;
    *nstreams = it->second.nstreams;
    *schedule = it->second.schedule;
    return true;
}

void clear_tuned() {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    g_tuned.clear();
    g_cache_loaded = false;
}

// Pipeline model of the staged path for N systems in batches of s, with
// N_b = ceil(N/s) batches and N_b + 2 pipeline steps (Algorithm 2): at step k
// Stage A of batch k, Stage B of batch k-1 and Stage C of batch k-2 are
// issued, when those batches exist.  concurrent = 0: the stages of a step run
// one after another (the comm-overlap-only schedule of the paper's estimator,
// which on one GPU has no communication to hide); concurrent = 1: Stage B
// runs beside A and C on its own stream (concurrent kernel execution), so a
// step costs max(A + C, B).
double pipeline_model_ms(int64_t N, int64_t s, double tA, double tB, double tC, int concurrent) {
    const int64_t nb = (N + s - 1) / s;
    double total = 0.0;
    for (int64_t k = 1; k <= nb + 2; ++k) {
        const double a = k <= nb ? tA : 0.0;
        const double b = (k >= 2 && k <= nb + 1) ? tB : 0.0;
        const double c = k >= 3 ? tC : 0.0;
        total += concurrent ? std::max(a + c, b) : a + b + c;
    }
    return total;
}

// Round-robin schedule (the pipeline's default): batch b runs A, B, C on
// stream b mod K, so the K streams run K batches at a time.  t1[] are the
// stage times of one batch alone, tK[] of K batches at once (one per
// stream); a full round of K batches costs tK[A] + tK[B] + tK[C], and the
// last, partial round of r batches costs max(t1, tK r / K) per stage (at
// least one batch's time, at most a full round's).  The remainder batch is
// costed at full size.
double round_robin_model_ms(int64_t nb, int K, const float *t1, const float *tK) {
    const int64_t rounds = nb / K, r = nb % K;
    double total = 0.0;
    for (int x = 0; x < 3; ++x) {
        total += (double)rounds * tK[x];
        if (r > 0) total += std::max((double)t1[x], (double)tK[x] * (double)r / K);
    }
    return total;
}

}  // namespace tdma

using namespace tdma;

extern "C" {

double tdma_pipeline_model_ms(int64_t nsys, int64_t batch, double t_a, double t_b, double t_c,
                              int concurrent) {
    if (nsys <= 0 || batch <= 0) return 0.0;
    return pipeline_model_ms(nsys, batch, t_a, t_b, t_c, concurrent);
}

const char *tdma_autotune_last_json(void) { return g_last_json.c_str(); }

int tdma_autotune(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype, const void *d,
                  void *x, int what, void *stream) {
    clear_error();
    int rc = validate(layout, coeffs, dtype, d, x);
    if (rc != TDMA_OK) return rc;
    if (layout->offsets) return fail(TDMA_EUNSUPPORTED, "autotune takes uniform layouts");
    if (what < 0 || what > 2) return fail(TDMA_EINVAL, "what = %d (0..2)", what);
    if (d == x) return fail(TDMA_EINVAL, "autotune overwrites x; it must not alias d");
    DeviceCtx *ctx = nullptr;
    rc = get_ctx(&ctx);
    if (rc != TDMA_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)stream;
    const int64_t nsys = layout->nsys0 * layout->nsys1;
    if (nsys == 0) return TDMA_OK;
    std::ostringstream js;
    if (what == 0) {
        std::vector<TileShape> cands = fused_candidates(dtype, layout, coeffs);
        if (cands.empty()) return fail(TDMA_EUNSUPPORTED, "no fused tile fits n = %lld", (long long)layout->n);
        float best = 1e30f;
        TileShape best_sh = cands[0];
        js << "{\"path\":\"fused\",\"candidates\":[";
        bool first = true;
        for (const TileShape &sh : cands) {
            float ms = 0.f;
            rc = time_median(st, 5, [&]() { return run_fused(ctx, layout, coeffs, dtype, d, x, st, &sh); }, &ms);
            if (rc != TDMA_OK) return rc;
            js << (first ? "" : ",") << "{\"kernel\":" << sh.kernel << ",\"M\":" << sh.M << ",\"S\":"
               << (1 << sh.S_log2) << ",\"P\":" << sh.P << ",\"ms\":" << ms << "}";
            first = false;
            if (ms < best) { best = ms; best_sh = sh; }
        }
        js << "],\"best\":{\"kernel\":" << best_sh.kernel << ",\"M\":" << best_sh.M << ",\"S\":"
           << (1 << best_sh.S_log2) << ",\"P\":" << best_sh.P << ",\"ms\":" << best << "}}";
        std::lock_guard<std::mutex> g(g_tune_mutex);
        load_cache_locked();
        Tuned &t = g_tuned[key_of(ctx->dev, layout, coeffs, dtype, "fused", 0)];
        t.shape = best_sh;
        t.has_shape = true;
        save_cache_locked();
        g_last_json = js.str();
        return TDMA_OK;
    }
    // staged path: every partition count P (powers of two, n/P >= 2) with
    // every batch size
    std::vector<int> Ps;
    for (int P = 2; P <= 32; P <<= 1)
        if (layout->n / P >= 2) Ps.push_back(P);
    if (Ps.empty()) return fail(TDMA_EINVAL, "n = %lld is too short to partition", (long long)layout->n);
    std::vector<int64_t> sizes;
    for (int64_t s = 1 << 12; s <= (1 << 18); s <<= 1) sizes.push_back(std::min(s, nsys));
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    const SysMap map = make_map(layout);
    const Coef coef = make_coef(coeffs);
    const bool shared_factors = coeffs->mode == TDMA_COEF_SHARED && coeffs->b_shift == nullptr;
    const size_t esz = dtype == TDMA_F64 ? 8 : 4;
    js << "{\"path\":\"partitioned\",\"streams\":" << kTuneStreams << ",\"candidates\":[";
    double best_model = 1e300, best_brute = 1e300;
    int64_t s_model = sizes[0], s_brute = sizes[0];
    int P_model = Ps[0], P_brute = Ps[0];
    std::vector<int64_t> per_P_batch(Ps.size(), sizes[0]);
    bool first = true;
    for (size_t pi = 0; pi < Ps.size(); ++pi) {
        const int P = Ps[pi];
        double best_model_P = 1e300;
        for (int64_t s : sizes) {
            const int64_t nb = (nsys + s - 1) / s;
            const int64_t nb_full = std::max<int64_t>(1, nsys / s);   // batches of exactly s systems
            const int K = (int)std::min<int64_t>(kTuneStreams, nb);
            // K batch workspaces (the layout of one pipeline slot each)
            const size_t fac = shared_factors ? (size_t)layout->n : (size_t)layout->n * s;
            const size_t fac_bytes = (fac * esz + 255) & ~(size_t)255;
            const size_t dh_bytes = ((size_t)layout->n * s * esz + 255) & ~(size_t)255;
            const size_t red_bytes = ((size_t)6 * P * s * 8 + 255) & ~(size_t)255;
            const size_t x_bytes = ((size_t)2 * P * s * 8 + 255) & ~(size_t)255;
            const size_t slot_bytes = dh_bytes + 2 * fac_bytes + red_bytes + 2 * x_bytes;
            void *ws = nullptr;
            rc = ctx->workspace(4, slot_bytes * K, &ws);
            if (rc != TDMA_OK) return rc;
            struct Slot { void *wd, *wa, *wc; double *red, *X, *scr; };
            std::vector<Slot> sl(K);
            for (int i = 0; i < K; ++i) {
                char *b = (char *)ws + slot_bytes * i;
                sl[i].wd = b;
                b += dh_bytes;
                sl[i].wa = b;
                sl[i].wc = b + fac_bytes;
                sl[i].red = (double *)(b + 2 * fac_bytes);
                sl[i].X = (double *)(b + 2 * fac_bytes + red_bytes);
                sl[i].scr = (double *)(b + 2 * fac_bytes + red_bytes + x_bytes);
            }
            // every repetition takes other batches (full ones, so each stage
            // reads what the previous stage wrote for it): a batch's data is
            // not left in the caches by the previous repetition
            int rep = 0;
            auto batch_of = [&](int r, int i) { return (((int64_t)r * K + i) % nb_full) * s; };
            auto stage = [&](int which, int i, int64_t k0, hipStream_t q) -> int {
                hipError_t e;
                if (which == 0)
                    e = launch_stage_a(dtype, map, coef, d, sl[i].wd, sl[i].wa, sl[i].wc, sl[i].red, k0, s,
                                       P, shared_factors, ctx->d_err, q);
                else if (which == 1)
                    e = launch_stage_b(sl[i].red, sl[i].X, sl[i].scr, s, P, ctx->d_err, q);
                else
                    e = launch_stage_c(dtype, map, x, sl[i].wd, sl[i].wa, sl[i].wc, sl[i].X, k0, s, P,
                                       shared_factors, q);
                return e == hipSuccess ? TDMA_OK : hip_fail(e, "autotune stage");
            };
            // one stage alone, and K instances of it at once on the pipeline's
            // streams (what the round-robin schedule runs)
            auto alone = [&](int which) {
                return [&, which]() { return stage(which, 0, batch_of(rep++, 0), st); };
            };
            auto together = [&](int which) {
                return [&, which]() -> int {
                    hipStream_t *qs = nullptr;
                    hipEvent_t *ev = nullptr;
                    int r2 = ctx->get_streams(K, &qs);
                    if (r2 == TDMA_OK) r2 = ctx->get_events(K + 1, &ev);
                    if (r2 != TDMA_OK) return r2;
                    hipError_t e = hipEventRecord(ev[0], st);
                    for (int i = 0; i < K && e == hipSuccess; ++i) e = hipStreamWaitEvent(qs[i], ev[0], 0);
                    if (e != hipSuccess) return hip_fail(e, "autotune fork");
                    for (int i = 0; i < K && r2 == TDMA_OK; ++i) r2 = stage(which, i, batch_of(rep, i), qs[i]);
                    ++rep;
                    for (int i = 0; i < K && e == hipSuccess && r2 == TDMA_OK; ++i) {
                        e = hipEventRecord(ev[1 + i], qs[i]);
                        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[1 + i], 0);
                    }
                    if (r2 == TDMA_OK && e != hipSuccess) r2 = hip_fail(e, "autotune join");
                    return r2;
                };
            };
            float t1[3] = {0, 0, 0}, tK[3] = {0, 0, 0};
            for (int which = 0; which < 3 && rc == TDMA_OK; ++which) rc = time_median(st, 5, alone(which), &t1[which]);
            for (int which = 0; which < 3 && rc == TDMA_OK; ++which) rc = time_median(st, 5, together(which), &tK[which]);
            if (rc != TDMA_OK) return rc;
            const double model = round_robin_model_ms(nb, K, t1, tK);
            const double model_alg2 = pipeline_model_ms(nsys, s, t1[0], t1[1], t1[2], 1);
            float brute = -1.f;
            if (what == 2) {
                rc = time_median(st, 5, [&]() {
                    return pipeline_solve(ctx, layout, coeffs, dtype, d, x, P, s, kTuneStreams, 1, st);
                }, &brute);
                if (rc != TDMA_OK) return rc;
                if (brute < best_brute) { best_brute = brute; s_brute = s; P_brute = P; }
            }
            if (model < best_model_P) { best_model_P = model; per_P_batch[pi] = s; }
            if (model < best_model) { best_model = model; s_model = s; P_model = P; }
            js << (first ? "" : ",") << "{\"P\":" << P << ",\"batch\":" << s << ",\"t_a_ms\":" << t1[0]
               << ",\"t_b_ms\":" << t1[1] << ",\"t_c_ms\":" << t1[2] << ",\"t_a_k_ms\":" << tK[0]
               << ",\"t_b_k_ms\":" << tK[1] << ",\"t_c_k_ms\":" << tK[2] << ",\"model_ms\":" << model
               << ",\"model_alg2_ms\":" << model_alg2 << ",\"measured_ms\":" << brute << "}";
            first = false;
        }
    }
    js << "],\"P\":" << P_model << ",\"model_choice\":" << s_model << ",\"model_ms\":" << best_model;
    if (what == 2)
        js << ",\"brute_choice_P\":" << P_brute << ",\"brute_choice\":" << s_brute
           << ",\"brute_ms\":" << best_brute;
    js << "}";
    std::lock_guard<std::mutex> g(g_tune_mutex);
    load_cache_locked();
    // the best batch of each P (for callers that fix P), and the overall
    // choice under P = 0 (for callers that leave P to the tuner)
    for (size_t pi = 0; pi < Ps.size(); ++pi) {
        Tuned &t = g_tuned[key_of(ctx->dev, layout, coeffs, dtype, "part", Ps[pi])];
        t.batch = per_P_batch[pi];
        t.nstreams = kTuneStreams;
        t.schedule = 1;   // round robin (the pipeline's numbering)
        t.P = Ps[pi];
    }
    Tuned &t = g_tuned[key_of(ctx->dev, layout, coeffs, dtype, "part", 0)];
    t.batch = s_model;
    t.nstreams = kTuneStreams;
    t.schedule = 1;
    t.P = P_model;
    save_cache_locked();
    g_last_json = js.str();
    return TDMA_OK;
}

}  // extern "C"
