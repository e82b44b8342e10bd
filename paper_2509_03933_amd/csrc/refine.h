// Device-side state of one tdma_solve_refined call (refine.hip / refine.cpp).
#pragma once
#include "tdma_internal.h"

namespace tdma {

struct RefineState {
    unsigned long long not_converged;  // systems whose last correction missed tol
    unsigned long long max_rel_bits;   // bits of the largest max|e|/max|x| (>= 0, so ordered)
    int32_t *fallback_list;            // ids of the systems that missed tol
    int64_t list_capacity;
};

size_t refine_lds_bytes(const TileShape &sh, bool like_d);
int refine_max_threads(int M);
bool refine_supported(const TileShape &sh, bool like_d);
hipError_t launch_refine(const SysMap &map, const Coef &coef, const TileShape &sh, const double *d,
                         double *x, int iters, double tol, RefineState *state, hipStream_t st);
hipError_t launch_refine_init(RefineState *state, int32_t *list, int64_t capacity, hipStream_t st);

// FP64 polishing of listed systems with double-double residuals (refine.hip)
int polish_partitions(int64_t n);
hipError_t launch_polish(const SysMap &map, const Coef &coef, const double *d, double *x,
                         const int32_t *list, const unsigned long long *count, int64_t capacity,
                         int steps, hipStream_t st);

// shared-operator variant (shared.hip)
size_t shared_refine_lds_bytes(const TileShape &sh);
bool shared_refine_supported(const TileShape &sh);
hipError_t launch_shared_refine(const SysMap &map, const Coef &coef, const TileShape &sh,
                                const double *d, double *x, int iters, double tol,
                                RefineState *state, hipStream_t st);

}  // namespace tdma
