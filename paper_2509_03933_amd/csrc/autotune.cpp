// Autotuner: tile shapes of the fused path, batch size of the staged path.
//
// Fused path: every applicable tile shape (kernel variant, rows per lane M,
// systems per tile S, partitions P) is timed with hipEvents on the caller's
// buffers; the fastest is cached for this shape.
//
// Staged path (the paper's batch-size optimisation, Sec. 4.2.3): for each
// partition count P (2..32, n/P >= 2) and each candidate batch size s
// (powers of two from 2^12 to 2^18, clipped to the number of systems) the
// mean time of Stage A, B and C on one batch is
// measured with each stage run alone, and the total is predicted from the
// pipelined schedule of Algorithm 2 with N_b = ceil(N/s) batches:
//     T(s) = sum_{k=1}^{N_b+2} max([k <= N_b] t_A + [k >= 3] t_C, [2 <= k <= N_b+1] t_B)
// i.e. Stage B overlapping A and C by concurrent kernel execution (one GPU
// has no communication stages, so the comm-overlap-only schedule of the
// paper's estimator would reduce to the plain sum of stage times, which is
// recorded too; the remainder batch is costed at full size).  The argmin is
// cached.  Mode 2
// also runs the full pipeline for every candidate (brute force) and records
// both, so the model's choice can be checked against the measured best.
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
                for (int kind : {1, 2}) {
                    TileShape sh;
                    sh.kernel = kind; sh.M = M; sh.P = P; sh.S_log2 = S_log2; sh.contig = contig;
                    if ((1 << S_log2) * P < 64 && (int64_t)(1 << S_log2) < nsys) continue;
                    if (shared_supported(dtype, sh)) out.push_back(sh);
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
    js << "{\"path\":\"partitioned\",\"candidates\":[";
    double best_model = 1e300, best_brute = 1e300;
    int64_t s_model = sizes[0], s_brute = sizes[0];
    int P_model = Ps[0], P_brute = Ps[0];
    std::vector<int64_t> per_P_batch(Ps.size(), sizes[0]);
    bool first = true;
    for (size_t pi = 0; pi < Ps.size(); ++pi) {
        const int P = Ps[pi];
        double best_model_P = 1e300;
        for (int64_t s : sizes) {
            // one batch worth of workspace (slot 0 of the pipeline workspace)
            const size_t fac = shared_factors ? (size_t)layout->n : (size_t)layout->n * s;
            const size_t fac_bytes = (fac * esz + 255) & ~(size_t)255;
            const size_t dh_bytes = ((size_t)layout->n * s * esz + 255) & ~(size_t)255;
            const size_t red_bytes = ((size_t)6 * P * s * 8 + 255) & ~(size_t)255;
            const size_t x_bytes = ((size_t)2 * P * s * 8 + 255) & ~(size_t)255;
            void *ws = nullptr;
            rc = ctx->workspace(4, dh_bytes + 2 * fac_bytes + red_bytes + 2 * x_bytes, &ws);
            if (rc != TDMA_OK) return rc;
            char *wd_ = (char *)ws;
            char *b = wd_ + dh_bytes;
            void *wa = b, *wc = b + fac_bytes;
            double *red = (double *)(b + 2 * fac_bytes), *X = (double *)(b + 2 * fac_bytes + red_bytes);
            double *scr = (double *)(b + 2 * fac_bytes + red_bytes + x_bytes);
            float tA = 0, tB = 0, tC = 0;
            rc = time_median(st, 3, [&]() {
                hipError_t e = launch_stage_a(dtype, map, coef, d, wd_, wa, wc, red, 0, s, P,
                                              shared_factors, ctx->d_err, st);
                return e == hipSuccess ? TDMA_OK : hip_fail(e, "stage A");
            }, &tA);
            if (rc == TDMA_OK) rc = time_median(st, 3, [&]() {
                hipError_t e = launch_stage_b(red, X, scr, s, P, ctx->d_err, st);
                return e == hipSuccess ? TDMA_OK : hip_fail(e, "stage B");
            }, &tB);
            if (rc == TDMA_OK) rc = time_median(st, 3, [&]() {
                hipError_t e = launch_stage_c(dtype, map, x, wd_, wa, wc, X, 0, s, P, shared_factors, st);
                return e == hipSuccess ? TDMA_OK : hip_fail(e, "stage C");
            }, &tC);
            if (rc != TDMA_OK) return rc;
            const double model = pipeline_model_ms(nsys, s, tA, tB, tC, 1);
            const double model_seq = pipeline_model_ms(nsys, s, tA, tB, tC, 0);
            float brute = -1.f;
            if (what == 2) {
                rc = time_median(st, 3, [&]() {
                    return pipeline_solve(ctx, layout, coeffs, dtype, d, x, P, s, 4, 1, st);
                }, &brute);
                if (rc != TDMA_OK) return rc;
                if (brute < best_brute) { best_brute = brute; s_brute = s; P_brute = P; }
            }
            if (model < best_model_P) { best_model_P = model; per_P_batch[pi] = s; }
            if (model < best_model) { best_model = model; s_model = s; P_model = P; }
            js << (first ? "" : ",") << "{\"P\":" << P << ",\"batch\":" << s << ",\"t_a_ms\":" << tA
               << ",\"t_b_ms\":" << tB << ",\"t_c_ms\":" << tC << ",\"model_ms\":" << model
               << ",\"model_sequential_ms\":" << model_seq << ",\"measured_ms\":" << brute << "}";
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
        t.nstreams = 4;
        t.schedule = 1;   // round robin (the pipeline's numbering)
        t.P = Ps[pi];
    }
    Tuned &t = g_tuned[key_of(ctx->dev, layout, coeffs, dtype, "part", 0)];
    t.batch = s_model;
    t.nstreams = 4;
    t.schedule = 1;
    t.P = P_model;
    save_cache_locked();
    g_last_json = js.str();
    return TDMA_OK;
}

}  // extern "C"
