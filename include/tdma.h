/*
 * tdma.h -- C ABI of the MI355X batched divide-and-conquer tridiagonal solver.
 *
 * Problem (paper, Algorithms 1 and 2, Sec. 3.2.1): the same tridiagonal solve
 * A x = d repeated for N independent systems, from the three diagonals a
 * (sub), b (main), c (super) and the right-hand side d to the solution x.  Each system is split into P partitions;
 * every partition is reduced by a modified Thomas sweep to two interface
 * equations (Stage A, Sec. 2.1 step 1), the 2P-row interface system is
 * solved (Stage B, step 3), and the interior unknowns are recovered from the
 * interface values (Stage C, step 5: x = x~ - Y y).
 *
 * General rules for every entry point:
 *  - Data pointers (a, b, c, b_shift, d, x) are DEVICE pointers owned by the
 *    caller; the library never frees or retains them past the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are stream-ordered and asynchronous unless stated otherwise.
 *  - x may alias d (in-place solve; tdma_solve_refined only without its
 *    FP64 fallback).  x must not alias a, b, c or b_shift.
 *  - a[0] and c[n-1] of every system are never read (no x_{-1}, no x_n).
 *  - No pivoting: results are defined for diagonally dominant systems and
 *    M-matrices (the paper's ADI and Poisson operators, Sec. 5).
 *  - Return value: a tdma_status.  Nothing is thrown across the ABI; details
 *    of the last failure on the calling thread are in tdma_last_error().
 *  - A zero or non-finite pivot met on the device sets a sticky per-device
 *    flag, reported as TDMA_ESINGULAR by tdma_check() (which clears it).
 *  - Element counts, strides and offsets are in ELEMENTS, not bytes.
 *  - One call takes at most 2^31 - 1 systems (TDMA_EUNSUPPORTED beyond; split
 *    the batch) and a layout spanning fewer than 2^62 elements (TDMA_EINVAL).
 *  - Threads: any host thread may call; each device's host-side state (plan
 *    cache, workspaces, stream and event pools) is locked for a call's host
 *    work.  The workspaces are per device, so tdma_solve_partitioned,
 *    tdma_solve_refined and tdma_autotune calls whose GPU work would overlap
 *    in time (different streams) must be ordered by the caller (same stream
 *    or events); tdma_solve_batched calls need no such ordering.
 *    tdma_shutdown must not overlap any other call.
 */
#ifndef TDMA_H
#define TDMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TDMA_OK = 0,
    TDMA_EINVAL = -1,        /* invalid argument (host-side validation)            */
    TDMA_ENOMEM = -2,        /* device or host allocation failed                   */
    TDMA_EHIP = -3,          /* a HIP runtime call failed                          */
    TDMA_ESINGULAR = -4,     /* zero or non-finite pivot met on the device         */
    TDMA_ENOCONV = -5,       /* refinement missed its tolerance (no fallback)      */
    TDMA_EUNSUPPORTED = -6   /* valid but unsupported combination                  */
} tdma_status;

typedef enum { TDMA_F64 = 0, TDMA_F32 = 1 } tdma_dtype;

typedef enum {
    TDMA_COEF_LIKE_D = 0,    /* a, b, c are laid out exactly like d (per-row)      */
    TDMA_COEF_SHARED = 1     /* a, b, c are length-n tables used by every system   */
} tdma_coef_mode;

/*
 * Where the systems live.  Uniform form (offsets == NULL): system
 * k = s0 + nsys0*s1 (0 <= s0 < nsys0, 0 <= s1 < nsys1) has its row i
 * (0 <= i < n) at element  s0*sys_stride0 + s1*sys_stride1 + i*row_stride.
 * This expresses the x-, y- and z-direction lines of a 3-D field (the
 * paper's assembly/reinsertion, Sec. 8.1) without copying.
 * Ragged form (offsets != NULL): `offsets` is a HOST array of nsys0+1
 * non-decreasing int64 entries, nsys1 must be 1, and system k occupies the
 * contiguous elements offsets[k] .. offsets[k+1]-1; `n` is ignored.
 * Every system needs n >= 2.  Ragged systems hold 2 .. 8192 rows in FP64 and
 * 2 .. 16384 in FP32 (longer systems: TDMA_EUNSUPPORTED).
 */
typedef struct tdma_layout {
    int64_t n;
    int64_t nsys0, nsys1;
    int64_t row_stride;
    int64_t sys_stride0, sys_stride1;
    const int64_t *offsets;
} tdma_layout;

/*
 * The coefficients.  mode TDMA_COEF_LIKE_D: a, b, c have d's layout.
 * mode TDMA_COEF_SHARED: a, b, c are contiguous length-n tables shared by
 * every system -- the paper's observation that the coefficient matrix
 * depends only on the grid spacing (Sec. 6.2.1); not allowed with offsets.
 * b_shift (optional, either mode): one value per system (index k as above)
 * added to every diagonal entry of that system, e.g. the -lambda of an
 * FFT-Poisson wavenumber (Sec. 5.2).  Same dtype as d.
 */
typedef struct tdma_coeffs {
    int mode;
    const void *a, *b, *c;
    const void *b_shift;
} tdma_coeffs;

/*
 * tdma_solve_batched: solve every system of `layout` in one fused launch.
 * Each system is split into P partitions held on chip (registers), reduced
 * by the modified Thomas sweep, the 2P-row interface system is solved in
 * FP64 by parallel cyclic reduction, and the interior is back-substituted;
 * only the inputs are read and x written (no intermediate HBM traffic).
 * dtype: TDMA_F64 (FP64 storage and sweeps) or TDMA_F32 (FP32 storage and
 * sweeps, FP64 interface solve).  The partition count and tile shape come
 * from the autotune cache if it holds this shape, else a built-in rule.
 * A ragged batch with per-row coefficients is one launch per block size (at
 * most two): its systems are grouped by the partition count they need and the
 * groups cut into tiles of one block each (a plan built on the first call
 * with these offsets and cached); otherwise it takes one launch per group.
 * A ragged layout on a stream that the caller is capturing into a graph is
 * refused with TDMA_EUNSUPPORTED (its plan tables are allocated and cached
 * by the library); tdma_graph_create records ragged solves instead.
 */
int tdma_solve_batched(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                       const void *d, void *x, void *stream);

/*
 * Explicit tile shape of the fused path (the autotuner's handle, also used by
 * tests).  kernel 0 (generic): rows_per_lane M = 4, 8, 16 (FP64) or 4, 8, 16,
 * 32 (FP32); systems_per_tile S a power of two; partitions P with M*P >= n;
 * S*P lanes form one workgroup, at most 1024 (512 when M rows of one array
 * fill 128 bytes).  kernel 1 (shared operator: TDMA_COEF_SHARED without
 * b_shift; coefficient factors built once per workgroup in LDS): M = 8, 12,
 * 16, 24, 32 and P a power of two <= 64; at most 1024 lanes, 512 when M
 * rows of one array fill 192 bytes.  kernel 2: kernel 1 in streaming form: as
 * many workgroups as fit the device at once each build the factors once and
 * walk the tiles, loading the next tile's right-hand sides while solving the
 * current one.  With contiguous rows it streams when the systems are
 * consecutive (system k at element k*n) and otherwise runs as kernel 1, with
 * the same results; with contiguous rows its lanes are capped at 512 when M
 * rows fill 128 bytes and 256 when they fill 256.  kernel 3 (shared operator
 * with b_shift, strided rows): M = 8, 16, 32, P a power of two <= 64, at most
 * 1024 lanes (512 at M = 32 in FP64); workgroups walk the tiles and load the
 * next tile's right-hand sides as the current one's rows are stored (when
 * P*M = n; otherwise as kernel 4).  kernel 4: kernel 3 loading each tile at
 * its start.  kernel 5 (per-row coefficients, TDMA_COEF_LIKE_D without
 * b_shift, strided rows): M = 16 or 32, P a power of two 2..64, at most 1024
 * lanes (512 at M = 32); workgroups walk the tiles, each lane
 * consuming its rows through a window of loads in flight.  kernel 6 (shared
 * operator without b_shift, strided rows): kernel 2 holding one set of
 * right-hand sides per lane, each register refilled with the next tile's row
 * as Stage C stores the current one (the row order alternating between
 * tiles), so that wider tiles fit: M*P = n exactly, at most 1024 lanes (512
 * when M rows fill 256 bytes); results equal kernel 2's.  kernel 7 (shared
 * operator with b_shift, strided rows, FP64): kernel 3 holding only the
 * right-hand sides, the pivots recomputed in Stage C, so that 32-system tiles
 * fit: M = 16 or 32, M*P = n exactly, at most 1024 lanes; results equal
 * kernel 3's.  Kernels 3-7 take fewer than 2^31 / 3 systems.  Uniform layouts
 * only.
 * Errors: EINVAL for a shape outside these rules or with M*P < n.
 */
typedef struct tdma_tile {
    int rows_per_lane;
    int systems_per_tile;
    int partitions;
    int kernel;
} tdma_tile;

int tdma_solve_batched_tiled(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                             const void *d, void *x, const tdma_tile *tile, void *stream);

/*
 * tdma_solve_pdd: the PDD approximation (Sun's parallel diagonally dominant
 * method; the paper solves its wall-normal momentum systems with it, Sec.
 * 5.1) in the fused kernel.  Each system is split into partitions of
 * rows_per_partition rows (the last one shorter); Stage A and C are those of
 * tdma_solve_batched, Stage B solves, for every pair of neighbouring
 * partitions, the 2 x 2 system of the last unknown of the one and the first
 * of the other, with the couplings to the far neighbours dropped (the spike
 * tips: for a diagonally dominant matrix they decay geometrically with the
 * partition length, and so does the error against the exact solution; the
 * caller chooses the length for the accuracy it needs).  One partition
 * (n <= rows_per_partition) gives the exact solution.
 * rows_per_partition: 4, 8 or 16 (FP64), also 32 (FP32); at most 1024
 * partitions (512 for 16 rows in FP64, 32 in FP32).  Any coefficient mode,
 * uniform layouts.  Errors: EINVAL for another partition length or a ragged
 * layout, EUNSUPPORTED for too many partitions.  x may alias d.
 */
int tdma_solve_pdd(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                   int rows_per_partition, const void *d, void *x, void *stream);

/*
 * The FFT-Poisson step (the paper's Poisson solve, Sec. 5.2): for a real
 * field q on an nx x ny x nz grid (x fastest, then y, then z; periodic in x
 * and y), phi solves  (Dxx + Dyy + Dz) phi = q  where Dxx, Dyy are the
 * periodic second differences whose Fourier symbols are the caller's shifts
 * and Dz the tridiagonal z operator (a, b, c; Neumann walls make mode (0, 0)
 * singular).  Steps: a batched real-to-complex 2-D FFT over (y, x) for every
 * z (hipFFT), one complex tridiagonal solve per wavenumber pair
 * (tdma_solve_multi, the real and imaginary parts as two right-hand sides,
 * diagonal b + shift[mode]), the inverse FFT.  Mode (0, 0) is solved with its
 * row 0 replaced by x_0 = d_0 (this fixes the additive constant).
 * tdma_poisson_create: a, b, c are HOST arrays of nz values (a[0], c[nz-1]
 * unused); shift is a HOST array of ny * (nx/2 + 1) values, mode (kx, ky) at
 * ky * (nx/2 + 1) + kx (the negated modified wavenumber, so that the mode's
 * operator is a, b + shift, c).  The plan owns two half-spectrum buffers of
 * nz * ny * (nx/2 + 1) complex doubles and the hipFFT plans; it is made on
 * the current device.  nz <= 1024.  Errors: EINVAL (arguments), EUNSUPPORTED
 * (nz > 1024), ENOMEM, EHIP (hipFFT).
 * tdma_poisson_solve: q and phi are DEVICE arrays of nx*ny*nz doubles; q may
 * be used as scratch by the forward transform (its content afterwards is
 * unspecified).  Stream-ordered; calls on one plan share its buffers and
 * must be ordered by the caller; the plan's device must be current (else
 * EINVAL).
 * tdma_poisson_destroy: synchronises the device, then frees the plan.
 */
typedef struct tdma_poisson tdma_poisson;
int tdma_poisson_create(int nx, int ny, int nz, const double *a, const double *b, const double *c,
                        const double *shift, tdma_poisson **out);
int tdma_poisson_solve(tdma_poisson *plan, const double *q, double *phi, void *stream);
void tdma_poisson_destroy(tdma_poisson *plan);

/*
 * tdma_solve_multi: several right-hand sides per system over one operator.
 * System k of `layout` has nrhs right-hand sides; right-hand side r has its
 * row i at element (start of system k) + i*row_stride + r*rhs_stride of d,
 * and its solution at the same element of x.  All of a system's right-hand
 * sides share its coefficients, which must be TDMA_COEF_SHARED tables
 * (b_shift optional, one value per system).  The paper's Poisson lines are
 * the case in mind (Sec. 5.2, 8.1): a real operator with complex data, i.e.
 * nrhs = 2 and rhs_stride = 1 over an array of interleaved (re, im) pairs,
 * every stride of the layout counted in real elements (twice the complex
 * index).  One fused launch per two right-hand sides: each lane runs the
 * operator's recurrences (pivots, a^, c^) of its rows once and the d^
 * recurrence per right-hand side; the interface system (FP64) is eliminated
 * once for all of them.  Same results as tdma_solve_batched on each
 * right-hand side, up to rounding order.
 * Limits: uniform layouts; n <= 1024 rows in FP64, 2048 in FP32
 * (TDMA_EUNSUPPORTED beyond, and for per-row coefficients).  Errors: EINVAL
 * for nrhs < 1, rhs_stride < 0, rhs_stride 0 with nrhs > 1, a ragged layout,
 * or a span of 2^62 elements or more.  x may alias d.  When nrhs >= 2,
 * rhs_stride is 1, every stride is even and d and x are aligned to a pair,
 * each row's two right-hand sides move as one vector access.
 */
int tdma_solve_multi(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype, int nrhs,
                     int64_t rhs_stride, const void *d, void *x, void *stream);

/*
 * tdma_copy_streamed (measurement): dst = src on every system row, moved
 * with the tile walk, lane-to-row mapping and register double-buffering of
 * the streaming shared-operator solve that tdma_solve_batched picks for this
 * layout, on the same number of workgroups, with no arithmetic.  It gives the
 * memory ceiling of that access pattern on the device, the figure against
 * which the solve's bandwidth is read.  Uniform strided layouts only
 * (row_stride != 1); src and dst are device arrays in the layout (elements
 * outside the systems are not touched) and must differ.  Stream-ordered.
 * Errors: EINVAL (NULL or equal pointers, bad layout or dtype),
 * EUNSUPPORTED (contiguous rows, ragged layouts, n > 2048, or a layout past
 * the walk's 32-bit system indices).
 */
int tdma_copy_streamed(const tdma_layout *layout, int dtype, const void *src, void *dst,
                       void *stream);

/*
 * Options of the split, pipelined solve.  Zero fields take defaults.
 *  partitions  P per system (>= 1, n/P >= 2); 0 = autotuned (cached) or 8.
 *  batch       systems per pipeline batch (the paper's batch_z, Sec. 4.2.1);
 *              0 = autotuned (cached) or 32768.
 *  nstreams    HIP streams the pipeline uses (1..8); 0 = autotuned or 4.
 *  schedule    0 = autotuned (cached) or round robin;
 *              1 = round robin (batch b runs A->B->C on stream b mod nstreams);
 *              2 = stage roles as in Algorithm 2 (Stage A and C on one stream
 *              role, Stage B on another, ordered by events).
 * Errors: EINVAL for P < 1, n/P < 2, P > 4096, nstreams > 8, schedule
 * outside 0..2 or a negative batch.
 */
typedef struct tdma_part_opts {
    int partitions;
    int64_t batch;
    int nstreams;
    int schedule;
} tdma_part_opts;

/*
 * tdma_solve_partitioned: the paper's staged method on one GPU.  Each
 * system is split into P partitions (the paper's slabs).  Stage A streams
 * every partition once and writes its two interface equations (6 values,
 * the paper's "6p") to a reduced buffer; Stage B solves the 2P-row reduced
 * systems (FP64, PCR across lanes); Stage C recomputes each partition's
 * interior from its two interface values.  Systems are grouped into batches
 * that are pipelined over HIP streams with events, three batches in flight
 * (Algorithm 2), so the low-occupancy Stage B overlaps the bandwidth-bound
 * Stages A and C.  Results do not depend on batch size, stream count or
 * schedule (bit-identical).  opts may be NULL.  Uniform layouts only.
 * The caller's stream waits for the whole pipeline before later work.
 */
int tdma_solve_partitioned(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                           const void *d, void *x, const tdma_part_opts *opts, void *stream);

/*
 * Options and report of the precision form (mixed-precision refinement).
 *  max_iters  refinement steps after the first FP32 solve, 0..3; the default
 *             (opts NULL) is 3.
 *  tol        a system has converged when its tested ratio is <= tol;
 *             default 1e-15.
 *  fallback   1 (default): systems that still miss tol are re-solved by the
 *             FP64 path; 0: they are counted and TDMA_ENOCONV is returned.
 *  criterion  the tested ratio.  0 (default): the last correction,
 *             max|dx_k| / max|x|.  1: the error left after the last step as
 *             the contraction observed between the last two refinement
 *             corrections predicts it, max|dx_k| q / (1 - q) / max|x| with
 *             q = max|dx_k| / max|dx_{k-1}| (q >= 1 never converges); it
 *             needs max_iters >= 2 and is criterion 0 below that.  It keeps
 *             systems that converge slowly but steadily (ill-conditioned
 *             ones) out of the FP64 fallback.  The ratio is an estimate:
 *             for a bar B on the error, tol = B/10 keeps a margin (at
 *             tol = B a Poisson mode was accepted at 1.02 B).
 */
typedef struct tdma_refine_opts {
    int max_iters;
    double tol;
    int fallback;
    int criterion;
} tdma_refine_opts;

typedef struct tdma_refine_report {
    int iterations;               /* refinement steps run (max over systems)       */
    int64_t not_converged;        /* systems whose tested ratio exceeded tol       */
    int64_t fallback_systems;     /* systems re-solved by the FP64 path            */
    double max_rel_correction;    /* max over systems of the tested ratio          */
} tdma_refine_report;

/*
 * tdma_solve_refined: FP64 in, FP64 out, FP32 sweeps.  Per tile, on chip:
 * x0 = solve32(d); then up to max_iters times r = d - A x (FP64),
 * x += solve32(r).  The interface (Stage B) solve is FP64 in every pass.
 * Coefficients, d and x are FP64.  With report != NULL the call
 * synchronises the stream and fills the report; with report == NULL it is
 * asynchronous and non-converged systems are handled per `fallback`.
 * x may alias d only with fallback = 0 (the FP64 fallback re-reads d after
 * x is written): with the fallback on, an aliased call is refused (EINVAL).
 */
int tdma_solve_refined(const tdma_layout *layout, const tdma_coeffs *coeffs, const double *d,
                       double *x, const tdma_refine_opts *opts, tdma_refine_report *report,
                       void *stream);

/*
 * tdma_solve_refined_noalloc: tdma_solve_refined for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results;
 * it calls no allocating routine.  Its device state (the refinement state,
 * the fallback's error flag and the fallback list) lives in a fixed
 * 262,400-byte array that every device the library runs on holds until the
 * process ends; its address is looked up once per device, on the device's
 * first call (devices 0..63).  Limit: at most 65,536 systems of a call can
 * be listed for the FP64 fallback (as in tdma_solve_refined); when more miss
 * tol the call returns TDMA_ENOCONV with the count.  Calls on one device
 * share the array and the last call's contents stay in it: calls that
 * overlap in time on one device (different streams, or host threads without
 * ordering) race and must be ordered by the caller.  Numerical errors of the
 * fallback (a zero or non-finite pivot) are returned as TDMA_ESINGULAR when
 * report != NULL; tdma_check does not see them.
 */
int tdma_solve_refined_noalloc(const tdma_layout *layout, const tdma_coeffs *coeffs,
                               const double *d, double *x, const tdma_refine_opts *opts,
                               tdma_refine_report *report, void *stream);

/*
 * Batching form: a list of solves recorded once into a hipGraph, replayed as
 * one submission by tdma_graph_launch.  Each item is planned and launched
 * exactly as tdma_solve_batched would (same kernels, tile shapes and
 * results, bit for bit).  An item with `after` >= 0 reads item `after`'s
 * output (e.g. the y-sweep of an ADI step reads the x-sweep's): such items
 * and the items they read run in item order on the graph's main branch,
 * ordered by graph edges; independent items (a ragged batch) run on a
 * parallel branch beside them.  All items share one dtype.  Pointers and the
 * ragged offsets' contents are captured at creation (the offsets are copied
 * to device memory the graph owns); the data pointers must stay valid while
 * the graph is used.  Destroy graphs before tdma_shutdown.
 * Errors: EINVAL for an invalid item (as tdma_solve_batched) or an `after`
 * that does not name an earlier item; EUNSUPPORTED for an item the fused
 * path cannot take; EHIP/ENOMEM from capture or allocation.  Numerical
 * errors of a replay are reported by tdma_check.
 */
typedef struct tdma_work_item {
    tdma_layout layout;
    tdma_coeffs coeffs;
    const void *d;
    void *x;
    int after;                    /* index of an earlier item this one reads, or -1 */
} tdma_work_item;

typedef struct tdma_graph tdma_graph;

int tdma_graph_create(const tdma_work_item *items, int nitems, int dtype, tdma_graph **out);
int tdma_graph_launch(tdma_graph *graph, void *stream);
void tdma_graph_destroy(tdma_graph *graph);

/*
 * tdma_autotune: time candidate tile shapes (fused path) or partition counts
 * and batch sizes (partitioned path: P = 2..32 with n/P >= 2, batches of
 * 2^12..2^18 systems, chosen by the pipeline model of Sec. 4.2.3) for this
 * shape on the calling device, store the winner in the in-process cache (and
 * in the file named by TDMA_CACHE, if set).  The partitioned path caches the
 * model's best batch for every P (used when the caller fixes P) and its best
 * (P, batch) overall (used when the caller leaves P at 0).  Synchronous.
 * The buffers must be valid inputs of that shape; x is overwritten and must
 * not alias d.
 * what: 0 = fused path, 1 = partitioned path (model), 2 = partitioned path
 * (model, then measured check of the model's choice against brute force).
 */
int tdma_autotune(const tdma_layout *layout, const tdma_coeffs *coeffs, int dtype,
                  const void *d, void *x, int what, void *stream);

/* JSON record of the last tdma_autotune call on any thread: every candidate
 * with its measured time (and, for the staged path, the per-stage times,
 * the model's prediction and, with what = 2, the measured pipeline time),
 * and the choice.  The string stays valid until the next tdma_autotune. */
const char *tdma_autotune_last_json(void);

/* The staged path's pipeline model (the paper's batch-size estimator,
 * Sec. 4.2.3, on one GPU): predicted time of nsys systems in batches of
 * `batch` from the per-batch stage times t_a, t_b, t_c (any unit) over the
 * N_b + 2 steps of Algorithm 2 (step k issues A of batch k, B of batch k-1,
 * C of batch k-2).  concurrent = 0: the stages of a step add up;
 * concurrent = 1: B overlaps A and C (a step costs max(A + C, B)). */
double tdma_pipeline_model_ms(int64_t nsys, int64_t batch, double t_a, double t_b, double t_c,
                              int concurrent);

/* Synchronise `stream`; return TDMA_ESINGULAR (and clear the flag) if any
 * kernel on this device met a zero or non-finite pivot, else TDMA_OK. */
int tdma_check(void *stream);

const char *tdma_status_string(int status);
const char *tdma_last_error(void);

/* Release every device resource the library holds (plans, workspaces,
 * streams, events) on all devices.  Optional; safe to call more than once. */
void tdma_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* TDMA_H */
