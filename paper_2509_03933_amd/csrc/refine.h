// Device-side state of one tdma_solve_refined call (refine.hip / refine.cpp).
#pragma once
#include "tdma_internal.h"

namespace tdma {

struct RefineState {
    unsigned long long not_converged;  // systems that missed tol
    unsigned long long max_rel_bits;   // bits of the largest tested ratio (>= 0, so ordered)
    int32_t *fallback_list;            // ids of the systems that missed tol
    int64_t list_capacity;
    int criterion;                     // 0: last correction, 1: contraction estimate
};

// The ratio a system's convergence is judged by, given the largest entries
// of its last two corrections (e, e_prev) and of its solution: criterion 0
// takes the last correction, e / max|x|; criterion 1 the remaining error
// that the observed contraction q = e / e_prev predicts, e q / (1 - q)
// (a geometric tail; q >= 1 never converges).  The contraction is observed
// between two refinement corrections only: the first solve is the whole
// solution, and its ratio to the first correction measured an error ten
// times the bar on a moderately conditioned Poisson mode, so with fewer
// than two steps criterion 1 is criterion 0.
__device__ inline double refine_ratio(int criterion, int iters, double e, double e_prev,
                                      double xmax) {
    double val = e;
    if (criterion == 1 && iters >= 2) {
        if (e_prev > 0.0) {
            const double q = e / e_prev;
            val = q < 1.0 ? e * q / (1.0 - q) : __builtin_huge_val();
        } else {
            val = e > 0.0 ? __builtin_huge_val() : 0.0;
        }
    }
    const double rel = xmax > 0.0 ? val / xmax : (val > 0.0 ? 1.0 : 0.0);
    return rel == rel ? rel : 1e300;
}

// The largest ratio into the state.  Atomics on one address serialise (about
// 12 ns each), so the current value is read first and most callers skip the
// atomic; a stale read only costs an extra atomic.
__device__ inline void fold_max_rel(RefineState *st, double rel) {
    if (!(rel > 0.0)) return;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(rel);
    if (bits > __hip_atomic_load(&st->max_rel_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&st->max_rel_bits, bits);
}

// Packing of a lane's two correction maxima (FP32 values) into one double
// slot of an LDS exchange.
__device__ inline double pack_e(float e, float e_prev) {
    return __hiloint2double(__float_as_int(e_prev), __float_as_int(e));
}
__device__ inline void unpack_e(double v, float &e, float &e_prev) {
    e = __int_as_float(__double2loint(v));
    e_prev = __int_as_float(__double2hiint(v));
}

size_t refine_lds_bytes(const TileShape &sh, bool like_d);
int refine_max_threads(int M);
bool refine_supported(const TileShape &sh, bool like_d);
hipError_t launch_refine(const SysMap &map, const Coef &coef, const TileShape &sh, const double *d,
                         double *x, int iters, double tol, RefineState *state, hipStream_t st);
// Resets the state (and zeroes *clear_err unless it is null) with a kernel,
// not a memset, so the call may be recorded into a graph.
hipError_t launch_refine_init(RefineState *state, int32_t *list, int64_t capacity, int criterion,
                              int *clear_err, hipStream_t st);

// FP64 polishing of listed systems with double-double residuals (refine.hip)
int polish_partitions(int64_t n);
hipError_t launch_polish(const SysMap &map, const Coef &coef, const double *d, double *x,
                         const int32_t *list, const unsigned long long *count, int64_t capacity,
                         int steps, hipStream_t st);

// shared operator + per-system shift, strided layouts (shifted.hip)
bool shift_refine_supported(const SysMap &map, const TileShape &sh);
hipError_t launch_shift_refine(const SysMap &map, const Coef &coef, const TileShape &sh,
                               const double *d, double *x, int iters, double tol,
                               RefineState *state, hipStream_t st);

// shared-operator variant (shared.hip)
size_t shared_refine_lds_bytes(const TileShape &sh);
bool shared_refine_supported(const TileShape &sh);
hipError_t launch_shared_refine(const SysMap &map, const Coef &coef, const TileShape &sh,
                                const double *d, double *x, int iters, double tol,
                                RefineState *state, hipStream_t st);

}  // namespace tdma
