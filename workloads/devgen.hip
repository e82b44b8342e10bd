// Device fill kernels of the seeded workload generator (gfx950).
//
// Bit-identical to workloads/rng.py and workloads/configs.py: the same
// counter-based SplitMix64 hash, the same FP64 operations in the same order,
// built with -ffp-contract=off so no multiply-add is fused.  This library
// holds no tridiagonal-solver arithmetic; it only fills input arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t finalise(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform(uint64_t seed, uint64_t stream, uint64_t index,
                                          double lo, double hi) {
    const uint64_t x = seed * 0xD1B54A32D192ED03ull + stream * 0x9E3779B97F4A7C15ull;
    const uint64_t z = finalise(index + x + 0x9E3779B97F4A7C15ull);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    const double span = hi - lo;
    return lo + span * u;
}

enum { ST_A = 1, ST_B = 2, ST_C = 3, ST_D = 4, ST_NOISE = 6 };

// z-systems of an nx*ny*nz grid (row = idx / plane), per-row random law.
__global__ void k_perrow_grid(uint64_t seed, int64_t plane, int64_t nrow, int64_t total,
                              double *a, double *b, double *c, double *d) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t row = idx / plane;
    double av = uniform(seed, ST_A, idx, -1.0, 1.0);
    double cv = uniform(seed, ST_C, idx, -1.0, 1.0);
    if (row == 0) av = 0.0;
    if (row == nrow - 1) cv = 0.0;
    const double extra = uniform(seed, ST_B, idx, 1.0, 2.0);
    const double bv = (fabs(av) + fabs(cv)) + extra;
    a[idx] = av;
    b[idx] = bv;
    c[idx] = cv;
    d[idx] = uniform(seed, ST_D, idx, -1.0, 1.0);
}

// Smooth separable field plus uniform noise: (sx[i]*sy[j])*cz[k] + U(-amp, amp).
__global__ void k_smooth(uint64_t seed, int64_t nx, int64_t ny, int64_t total, const double *sx,
                         const double *sy, const double *cz, double amp, double *d) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t i = idx % nx;
    const int64_t j = (idx / nx) % ny;
    const int64_t k = idx / (nx * ny);
    const double noise = uniform(seed, ST_NOISE, idx, -amp, amp);
    d[idx] = (sx[i] * sy[j]) * cz[k] + noise;
}

// d ~ U(-1, 1), with element `pin` (if >= 0) set to zero.
__global__ void k_uniform_d(uint64_t seed, int64_t total, int64_t pin, double *d) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const double v = uniform(seed, ST_D, idx, -1.0, 1.0);
    d[idx] = (idx == pin) ? 0.0 : v;
}

inline unsigned blocks_for(int64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

extern "C" {

int wl_perrow_grid(uint64_t seed, int64_t plane, int64_t nrow, int64_t total, double *a, double *b,
                   double *c, double *d, void *stream) {
    if (total <= 0) return 0;
    hipLaunchKernelGGL(k_perrow_grid, dim3(blocks_for(total)), dim3(256), 0, (hipStream_t)stream,
                       seed, plane, nrow, total, a, b, c, d);
    return (int)hipGetLastError();
}

int wl_smooth(uint64_t seed, int64_t nx, int64_t ny, int64_t total, const double *sx,
              const double *sy, const double *cz, double amp, double *d, void *stream) {
    if (total <= 0) return 0;
    hipLaunchKernelGGL(k_smooth, dim3(blocks_for(total)), dim3(256), 0, (hipStream_t)stream, seed,
                       nx, ny, total, sx, sy, cz, amp, d);
    return (int)hipGetLastError();
}

int wl_uniform_d(uint64_t seed, int64_t total, int64_t pin, double *d, void *stream) {
    if (total <= 0) return 0;
    hipLaunchKernelGGL(k_uniform_d, dim3(blocks_for(total)), dim3(256), 0, (hipStream_t)stream,
                       seed, total, pin, d);
    return (int)hipGetLastError();
}

}  // extern "C"
