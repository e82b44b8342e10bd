// The FFT-Poisson step (the paper's Poisson solve, Sec. 5.2): a real field
// on an nx x ny x nz grid, periodic in x and y, is transformed in (y, x) by a
// batched real-to-complex 2-D FFT (hipFFT, one transform per z plane), every
// wavenumber pair's z-line -- a tridiagonal system with the z operator plus
// the mode's diagonal shift and a complex right-hand side -- is solved by the
// multi-right-hand-side kernel (real and imaginary parts as two right-hand
// sides), and the inverse 2-D FFT returns the field.  The inverse transform
// is unnormalised, so the operator tables are stored multiplied by nx*ny
// (x = (N A)^-1 d = A^-1 d / N): no scaling pass.  Mode (0, 0) is singular
// with Neumann walls; it is solved separately with its row 0 replaced by
// x_0 = d_0 (the bulk call gives it a placeholder shift and its result is
// overwritten).
#include <hipfft/hipfft.h>

#include <vector>

#include "api_internal.h"

struct tdma_poisson {
    int nx = 0, ny = 0, nz = 0, h = 0;
    int dev = 0;
    hipfftHandle fwd = 0, inv = 0;
    bool has_fwd = false, has_inv = false;
    double *W1 = nullptr, *W2 = nullptr;   // half spectra, (nz, ny, h) interleaved complex
    double *tab = nullptr;                 // a, b, c, pinned a, b, c (nz each), shift (ny*h)
};

using namespace tdma;

namespace {

void release(tdma_poisson *pl) {
    if (!pl) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(pl->dev);
    (void)hipDeviceSynchronize();   // no launch of this plan is still running
    if (pl->has_fwd) (void)hipfftDestroy(pl->fwd);
    if (pl->has_inv) (void)hipfftDestroy(pl->inv);
    if (pl->W1) (void)hipFree(pl->W1);
    if (pl->W2) (void)hipFree(pl->W2);
    if (pl->tab) (void)hipFree(pl->tab);
    (void)hipSetDevice(cur);
    delete pl;
}

int fft_fail(hipfftResult r, const char *what) {
    return fail(TDMA_EHIP, "%s failed (hipfftResult %d)", what, (int)r);
}

}  // namespace

extern "C" {

int tdma_poisson_create(int nx, int ny, int nz, const double *a, const double *b, const double *c,
                        const double *shift, tdma_poisson **out) {
    clear_error();
    if (!out) return fail(TDMA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!a || !b || !c || !shift) return fail(TDMA_EINVAL, "a, b, c and shift must be non-NULL");
    if (nx < 1 || ny < 1 || nz < 2) return fail(TDMA_EINVAL, "grid %d x %d x %d (nz >= 2)", nx, ny, nz);
    if (nz > 1024)
        return fail(TDMA_EUNSUPPORTED, "nz = %d is longer than the 1024 rows of the z solve", nz);
    if ((int64_t)nx * ny > (int64_t)1 << 30)
        return fail(TDMA_EUNSUPPORTED, "a %d x %d plane is larger than 2^30 points", nx, ny);
    tdma_poisson *pl = new tdma_poisson;
    pl->nx = nx;
    pl->ny = ny;
    pl->nz = nz;
    pl->h = nx / 2 + 1;
    hipError_t e = hipGetDevice(&pl->dev);
    if (e != hipSuccess) { delete pl; return hip_fail(e, "hipGetDevice"); }
    const int64_t modes = (int64_t)ny * pl->h;
    const double N = (double)nx * (double)ny;
    // tables scaled by N; the pinned set has row 0 = (0, N, 0); mode (0, 0)
    // takes another mode's shift in the bulk call (a placeholder)
    std::vector<double> t(6 * (size_t)nz + (size_t)modes);
    for (int k = 0; k < nz; ++k) {
        t[k] = N * a[k];
        t[nz + k] = N * b[k];
        t[2 * nz + k] = N * c[k];
        t[3 * nz + k] = N * a[k];
        t[4 * nz + k] = N * b[k];
        t[5 * nz + k] = N * c[k];
    }
    t[3 * nz] = 0.0;
    t[4 * nz] = N;
    t[5 * nz] = 0.0;
    for (int64_t m = 0; m < modes; ++m) t[6 * (size_t)nz + m] = N * shift[m];
    if (modes > 1) t[6 * (size_t)nz] = t[6 * (size_t)nz + 1];
    else t[6 * (size_t)nz] = -N;
    const size_t spec = (size_t)nz * modes * 2 * sizeof(double);
    if (hipMalloc(&pl->tab, t.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&pl->W1, spec) != hipSuccess || hipMalloc(&pl->W2, spec) != hipSuccess) {
        release(pl);
        return fail(TDMA_ENOMEM, "device buffers of the Poisson plan (%zu bytes each)", spec);
    }
    e = hipMemcpy(pl->tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) { release(pl); return hip_fail(e, "upload of the Poisson tables"); }
    int n[2] = {ny, nx};
    hipfftResult r = hipfftPlanMany(&pl->fwd, 2, n, nullptr, 1, nx * ny, nullptr, 1, (int)modes,
                                    HIPFFT_D2Z, nz);
    if (r != HIPFFT_SUCCESS) { release(pl); return fft_fail(r, "forward plan"); }
    pl->has_fwd = true;
    r = hipfftPlanMany(&pl->inv, 2, n, nullptr, 1, (int)modes, nullptr, 1, nx * ny, HIPFFT_Z2D, nz);
    if (r != HIPFFT_SUCCESS) { release(pl); return fft_fail(r, "inverse plan"); }
    pl->has_inv = true;
    *out = pl;
    return TDMA_OK;
}

int tdma_poisson_solve(tdma_poisson *pl, const double *q, double *phi, void *stream) {
    clear_error();
    if (!pl || !q || !phi) return fail(TDMA_EINVAL, "plan, q and phi must be non-NULL");
    int cur = -1;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != pl->dev)
        return fail(TDMA_EINVAL, "the plan was made on device %d, device %d is current", pl->dev, cur);
    const hipStream_t st = (hipStream_t)stream;
    const int nz = pl->nz, h = pl->h;
    hipfftResult r = hipfftSetStream(pl->fwd, st);
    if (r == HIPFFT_SUCCESS)
        r = hipfftExecD2Z(pl->fwd, const_cast<double *>(q), reinterpret_cast<hipfftDoubleComplex *>(pl->W1));
    if (r != HIPFFT_SUCCESS) return fft_fail(r, "forward transform");
    tdma_layout L{};
    L.n = nz;
    L.nsys0 = h;
    L.nsys1 = pl->ny;
    L.row_stride = 2 * (int64_t)pl->ny * h;
    L.sys_stride0 = 2;
    L.sys_stride1 = 2 * (int64_t)h;
    L.offsets = nullptr;
    tdma_coeffs C{};
    C.mode = TDMA_COEF_SHARED;
    C.a = pl->tab;
    C.b = pl->tab + nz;
    C.c = pl->tab + 2 * nz;
    C.b_shift = pl->tab + 6 * (size_t)nz;
    int rc = tdma_solve_multi(&L, &C, TDMA_F64, 2, 1, pl->W1, pl->W2, stream);
    if (rc != TDMA_OK) return rc;
    tdma_layout L0 = L;
    L0.nsys0 = 1;
    L0.nsys1 = 1;
    tdma_coeffs C0{};
    C0.mode = TDMA_COEF_SHARED;
    C0.a = pl->tab + 3 * nz;
    C0.b = pl->tab + 4 * nz;
    C0.c = pl->tab + 5 * nz;
    C0.b_shift = nullptr;
    rc = tdma_solve_multi(&L0, &C0, TDMA_F64, 2, 1, pl->W1, pl->W2, stream);
    if (rc != TDMA_OK) return rc;
    clear_error();
    r = hipfftSetStream(pl->inv, st);
    if (r == HIPFFT_SUCCESS)
        r = hipfftExecZ2D(pl->inv, reinterpret_cast<hipfftDoubleComplex *>(pl->W2), phi);
    if (r != HIPFFT_SUCCESS) return fft_fail(r, "inverse transform");
    return TDMA_OK;
}

void tdma_poisson_destroy(tdma_poisson *pl) { release(pl); }

}  // extern "C"
