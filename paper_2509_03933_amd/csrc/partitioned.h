// Launchers of the staged (split) path, partitioned.hip.
#pragma once
#include "tdma_internal.h"

namespace tdma {

hipError_t launch_stage_a(int dtype, const SysMap &map, const Coef &coef, const void *d,
                          void *ws_d, void *ws_a, void *ws_c, double *red, int64_t k_begin,
                          int64_t nb, int P, bool shared_factors, int *err, hipStream_t st);
hipError_t launch_stage_b(const double *red, double *X, double *scratch, int64_t nb, int P,
                          int *err, hipStream_t st);
hipError_t launch_stage_c(int dtype, const SysMap &map, void *x, const void *ws_d,
                          const void *ws_a, const void *ws_c, const double *X, int64_t k_begin,
                          int64_t nb, int P, bool shared_factors, hipStream_t st);

}  // namespace tdma
