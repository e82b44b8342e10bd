// Host-side internals shared by the API translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "tdma_internal.h"

namespace tdma {

constexpr int64_t kMaxRaggedRows = 16384;   // FP64 ragged systems stop at 8192

struct RaggedBucket {
    TileShape shape;
    int64_t first = 0;   // index into the device system list
    int64_t count = 0;
};

// Tiles of one rows-per-lane class in the single-launch form.
struct RaggedGroup {
    int M = 0;
    int threads = 0;
    size_t lds = 0;
    int64_t first_tile = 0, ntiles = 0;
};

struct RaggedPlan {
    int64_t nsys = 0;
    int dtype = -1;
    std::vector<int64_t> offsets;   // host copy: the plan cache compares it in full
    int64_t *d_offsets = nullptr;
    int32_t *d_list = nullptr;
    std::vector<RaggedBucket> buckets;
    // per-row coefficients: the buckets of one M and one block size in one
    // launch (tile list, longest systems first); empty when a tile would not
    // fit
    std::vector<RaggedGroup> groups;
    RaggedTile *d_tiles = nullptr;
};

struct Workspace {
    int slot = 0;
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct DeviceCtx {
    // guards the host-side state below (plan cache, workspaces, stream and
    // event pools); every entry point holds it for its host work
    std::mutex mu;
    int dev = 0;
    int num_cus = 256;
    int *d_err = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<Workspace> workspaces;
    std::map<uint64_t, RaggedPlan> ragged_cache;
    ~DeviceCtx();
    void release();
    int workspace(int slot, size_t bytes, void **out);
    int get_streams(int count, hipStream_t **out);
    int get_events(int count, hipEvent_t **out);
};

int fail(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();
int get_ctx(DeviceCtx **out);
int validate(const tdma_layout *L, const tdma_coeffs *C, int dtype, const void *d, const void *x);
SysMap make_map(const tdma_layout *L);
Coef make_coef(const tdma_coeffs *C);
bool default_shape(int dtype, int64_t n, int64_t nsys, bool contig, TileShape *out);
// min_block: the smallest block of the per-row tile list (lanes): 256 for a
// batch solved on its own (two blocks share a CU), the kernel's largest block
// (0 = that) for a batch that runs beside other work, as in a graph.
int build_ragged_plan(const tdma_layout *L, int dtype, RaggedPlan *out, int min_block = 256);
void free_ragged_plan(RaggedPlan *rp);
int plan_ragged(DeviceCtx *ctx, const tdma_layout *L, int dtype, const RaggedPlan **out);
// The buckets of a ragged plan on st and up to naux streams aux at once
// (forked from st by event ev[0], joined back by ev[1..naux]); naux = 0
// keeps them all on st (the form recorded into graphs).
constexpr int kRaggedAux = 3;
int launch_ragged(const RaggedPlan &rp, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                  const void *d, void *x, int *err, hipStream_t st, const hipStream_t *aux,
                  int naux, const hipEvent_t *ev);
int plan_uniform(DeviceCtx *ctx, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                 const TileShape *force, TileShape *out);
int launch_uniform(const TileShape &sh, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                   const void *d, void *x, int *err, hipStream_t st);
int run_fused(DeviceCtx *ctx, const tdma_layout *L, const tdma_coeffs *C, int dtype, const void *d,
              void *x, hipStream_t st, const TileShape *force);

// autotune cache (autotune.cpp)
bool lookup_tuned(int dev, const tdma_layout *L, const tdma_coeffs *C, int dtype, TileShape *out);
// Tuned staged-path settings for partition count *P; *P = 0 asks for the
// tuner's own choice of P, which is written back.
bool lookup_tuned_batch(int dev, const tdma_layout *L, const tdma_coeffs *C, int dtype, int *P,
                        int64_t *batch, int *nstreams, int *schedule);
int pipeline_solve(DeviceCtx *ctx, const tdma_layout *L, const tdma_coeffs *C, int dtype,
                   const void *d, void *x, int P, int64_t batch, int nstreams, int schedule,
                   hipStream_t caller);
void clear_tuned();

}  // namespace tdma
