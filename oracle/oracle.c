/*
 * Oracle: plain, slow, obviously correct CPU solver for batches of
 * independent tridiagonal systems.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the GPU library.
 *
 * What it computes: x = A^{-1} d for every system, where A is tridiagonal
 * with sub-diagonal a, diagonal b and super-diagonal c (the problem of the
 * paper's Algorithms 1 and 2: N independent systems, from the three diagonals
 * and the right-hand side to the solution).  The divide-and-conquer method of the paper (Sec. 2.1: decoupled
 * solve, reduced interface solve, correction x = x~ - Y y) is a direct method
 * that reaches exactly this x in exact arithmetic, so the oracle is that
 * definition computed by the textbook Thomas algorithm (LU factorisation
 * without pivoting, forward elimination then back substitution; the
 * sequential O(n) method the paper's introduction starts from).
 *
 * Also here: the same definition for complex systems (oracle_thomas_z and its
 * batch over shared real tables, for the complex Poisson right-hand sides),
 * and the PDD approximation (oracle_pdd), which is not x = A^{-1} d but the
 * published partitioned method the paper uses for its momentum systems; its
 * header states its steps.
 *
 * Conventions: a[0] and c[n-1] of every system are never read (there is no
 * x_{-1} or x_n).  Arithmetic is IEEE FP64 (or x87 80-bit long double for the
 * *_ld variant), round to nearest, no fused multiply-add (built with
 * -ffp-contract=off), no fast-math.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_ESINGULAR (-4)

/* Thomas algorithm, FP64.  cp/dp are caller scratch of length n.
 * Forward:  c'_0 = c_0/b_0, d'_0 = d_0/b_0;
 *           m_i = b_i - a_i c'_{i-1}, c'_i = c_i/m_i, d'_i = (d_i - a_i d'_{i-1})/m_i.
 * Backward: x_{n-1} = d'_{n-1}, x_i = d'_i - c'_i x_{i+1}. */
static int thomas_f64(int64_t n, const double *a, const double *b, const double *c,
                      const double *d, double *x, double *cp, double *dp)
{
    double m = b[0];
    if (m == 0.0 || !isfinite(m)) return ORACLE_ESINGULAR;
    cp[0] = (n > 1) ? c[0] / m : 0.0;
    dp[0] = d[0] / m;
    for (int64_t i = 1; i < n; ++i) {
        m = b[i] - a[i] * cp[i - 1];
        if (m == 0.0 || !isfinite(m)) return ORACLE_ESINGULAR;
        cp[i] = (i < n - 1) ? c[i] / m : 0.0;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    return ORACLE_OK;
}

/* The same algorithm carried out in long double (x87 extended precision); the
 * result is rounded to double once at the end.  Used to tell the oracle's own
 * rounding apart from a candidate's error on ill-conditioned systems. */
static int thomas_ld(int64_t n, const double *a, const double *b, const double *c,
                     const double *d, double *x, long double *cp, long double *dp)
{
    long double m = b[0];
    if (m == 0.0L || !isfinite((double)m)) return ORACLE_ESINGULAR;
    cp[0] = (n > 1) ? (long double)c[0] / m : 0.0L;
    dp[0] = (long double)d[0] / m;
    for (int64_t i = 1; i < n; ++i) {
        m = (long double)b[i] - (long double)a[i] * cp[i - 1];
        if (m == 0.0L || !isfinite((double)m)) return ORACLE_ESINGULAR;
        cp[i] = (i < n - 1) ? (long double)c[i] / m : 0.0L;
        dp[i] = ((long double)d[i] - (long double)a[i] * dp[i - 1]) / m;
    }
    long double xn = dp[n - 1];
    x[n - 1] = (double)xn;
    /* keep the running x in long double: x_i = d'_i - c'_i x_{i+1} */
    for (int64_t i = n - 2; i >= 0; --i) {
        xn = dp[i] - cp[i] * xn;
        x[i] = (double)xn;
    }
    return ORACLE_OK;
}

/* One contiguous system. precision: 0 = FP64, 1 = long double. */
int oracle_thomas(int64_t n, const double *a, const double *b, const double *c,
                  const double *d, double *x, int precision)
{
    if (n < 1 || !a || !b || !c || !d || !x) return ORACLE_EINVAL;
    int rc;
    if (precision == 0) {
        double *w = (double *)malloc(2 * (size_t)n * sizeof(double));
        if (!w) return ORACLE_ENOMEM;
        rc = thomas_f64(n, a, b, c, d, x, w, w + n);
        free(w);
    } else {
        long double *w = (long double *)malloc(2 * (size_t)n * sizeof(long double));
        if (!w) return ORACLE_ENOMEM;
        rc = thomas_ld(n, a, b, c, d, x, w, w + n);
        free(w);
    }
    return rc;
}

/*
 * A batch of systems in a strided or ragged layout.  Each system is gathered
 * into contiguous arrays, solved by oracle_thomas, and its x scattered back.
 *
 * Uniform layout (offsets == NULL): system s = s0 + nsys0*s1 has row i at
 *     s0*sys_stride0 + s1*sys_stride1 + i*row_stride        (element units)
 * Ragged layout: system s (0 <= s < nsys0, nsys1 == 1) occupies elements
 *     offsets[s] .. offsets[s+1]-1, one row each.
 * coef_mode 0: a, b, c have d's layout.  coef_mode 1: a, b, c are length-n
 *     tables shared by every system; shift (may be NULL) adds shift[s] to
 *     every diagonal entry of system s.
 * Systems whose solve fails are reported through status[s] (may be NULL);
 * the return value is the number of failed systems, or a negative error.
 * sys_begin/sys_end restrict the solve to a range of system indices.
 */
int64_t oracle_solve_batch(int64_t n, int64_t nsys0, int64_t nsys1, int64_t row_stride,
                           int64_t sys_stride0, int64_t sys_stride1, const int64_t *offsets,
                           int coef_mode, const double *a, const double *b, const double *c,
                           const double *shift, const double *d, double *x,
                           int precision, int64_t sys_begin, int64_t sys_end, int32_t *status)
{
    if (!a || !b || !c || !d || !x) return ORACLE_EINVAL;
    if (offsets && nsys1 != 1) return ORACLE_EINVAL;
    if (offsets && coef_mode != 0) return ORACLE_EINVAL;
    int64_t nsys = nsys0 * nsys1;
    if (sys_begin < 0 || sys_end > nsys || sys_begin > sys_end) return ORACLE_EINVAL;
    int64_t nmax = n;
    if (offsets) {
        nmax = 0;
        for (int64_t s = sys_begin; s < sys_end; ++s)
            if (offsets[s + 1] - offsets[s] > nmax) nmax = offsets[s + 1] - offsets[s];
    }
    if (nmax < 1) return (sys_end > sys_begin) ? ORACLE_EINVAL : 0;
    double *buf = (double *)malloc(5 * (size_t)nmax * sizeof(double));
    int64_t *rows = (int64_t *)malloc((size_t)nmax * sizeof(int64_t));
    if (!buf || !rows) { free(buf); free(rows); return ORACLE_ENOMEM; }
    double *sa = buf, *sb = buf + nmax, *sc = buf + 2 * nmax, *sd = buf + 3 * nmax,
           *sx = buf + 4 * nmax;
    int64_t failed = 0;
    for (int64_t s = sys_begin; s < sys_end; ++s) {
        int64_t ns;
        if (offsets) {
            ns = offsets[s + 1] - offsets[s];
            for (int64_t i = 0; i < ns; ++i) rows[i] = offsets[s] + i;
        } else {
            ns = n;
            int64_t s0 = s % nsys0, s1 = s / nsys0;
            int64_t base = s0 * sys_stride0 + s1 * sys_stride1;
            for (int64_t i = 0; i < ns; ++i) rows[i] = base + i * row_stride;
        }
        for (int64_t i = 0; i < ns; ++i) {
            sd[i] = d[rows[i]];
            if (coef_mode == 0) {
                sa[i] = a[rows[i]];
                sb[i] = b[rows[i]];
                sc[i] = c[rows[i]];
            } else {
                sa[i] = a[i];
                sb[i] = shift ? b[i] + shift[s] : b[i];
                sc[i] = c[i];
            }
        }
        int rc = ns > 0 ? oracle_thomas(ns, sa, sb, sc, sd, sx, precision) : ORACLE_OK;
        if (status) status[s] = rc;
        if (rc != ORACLE_OK) { ++failed; continue; }
        for (int64_t i = 0; i < ns; ++i) x[rows[i]] = sx[i];
    }
    free(buf);
    free(rows);
    return failed;
}

/*
 * Complex systems (the paper's Poisson data are complex, Sec. 8.1): the same
 * Thomas recurrences with every quantity complex, in C99 complex arithmetic
 * (double complex, or long double complex for the extended variant).  Arrays
 * hold n interleaved (real, imaginary) pairs, the layout C gives a complex
 * array.  A zero or non-finite pivot fails the system.
 */
static int zbad(double complex m)
{
    return (creal(m) == 0.0 && cimag(m) == 0.0) || !isfinite(creal(m)) || !isfinite(cimag(m));
}

static int thomas_z(int64_t n, const double complex *a, const double complex *b,
                    const double complex *c, const double complex *d, double complex *x,
                    double complex *cp, double complex *dp)
{
    double complex m = b[0];
    if (zbad(m)) return ORACLE_ESINGULAR;
    cp[0] = (n > 1) ? c[0] / m : 0.0;
    dp[0] = d[0] / m;
    for (int64_t i = 1; i < n; ++i) {
        m = b[i] - a[i] * cp[i - 1];
        if (zbad(m)) return ORACLE_ESINGULAR;
        cp[i] = (i < n - 1) ? c[i] / m : 0.0;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    return ORACLE_OK;
}

static int thomas_zld(int64_t n, const double complex *a, const double complex *b,
                      const double complex *c, const double complex *d, double complex *x,
                      long double complex *cp, long double complex *dp)
{
    long double complex m = b[0];
    if (zbad((double complex)m)) return ORACLE_ESINGULAR;
    cp[0] = (n > 1) ? (long double complex)c[0] / m : 0.0L;
    dp[0] = (long double complex)d[0] / m;
    for (int64_t i = 1; i < n; ++i) {
        m = (long double complex)b[i] - (long double complex)a[i] * cp[i - 1];
        if (zbad((double complex)m)) return ORACLE_ESINGULAR;
        cp[i] = (i < n - 1) ? (long double complex)c[i] / m : 0.0L;
        dp[i] = ((long double complex)d[i] - (long double complex)a[i] * dp[i - 1]) / m;
    }
    long double complex xn = dp[n - 1];
    x[n - 1] = (double complex)xn;
    for (int64_t i = n - 2; i >= 0; --i) {
        xn = dp[i] - cp[i] * xn;
        x[i] = (double complex)xn;
    }
    return ORACLE_OK;
}

/* One complex system; a, b, c, d, x each hold n (re, im) pairs.
 * precision: 0 = FP64, 1 = long double. */
int oracle_thomas_z(int64_t n, const double *a, const double *b, const double *c,
                    const double *d, double *x, int precision)
{
    if (n < 1 || !a || !b || !c || !d || !x) return ORACLE_EINVAL;
    int rc;
    if (precision == 0) {
        double complex *w = (double complex *)malloc(2 * (size_t)n * sizeof(double complex));
        if (!w) return ORACLE_ENOMEM;
        rc = thomas_z(n, (const double complex *)a, (const double complex *)b,
                      (const double complex *)c, (const double complex *)d, (double complex *)x,
                      w, w + n);
        free(w);
    } else {
        long double complex *w =
            (long double complex *)malloc(2 * (size_t)n * sizeof(long double complex));
        if (!w) return ORACLE_ENOMEM;
        rc = thomas_zld(n, (const double complex *)a, (const double complex *)b,
                        (const double complex *)c, (const double complex *)d, (double complex *)x,
                        w, w + n);
        free(w);
    }
    return rc;
}

/*
 * A batch of complex systems over shared REAL coefficient tables a, b, c
 * (length n) with an optional real per-system diagonal shift -- the Poisson
 * line solves of Sec. 5.2 after the Fourier transform in x and y, whose
 * right-hand sides are complex.  Layout as in oracle_solve_batch, counted in
 * COMPLEX elements: d and x are interleaved (re, im) arrays.  Each system is
 * gathered, its coefficients widened to complex, solved by oracle_thomas_z and
 * scattered back.  Returns the number of failed systems (status[s] per
 * system, may be NULL) or a negative error.
 */
int64_t oracle_solve_batch_z(int64_t n, int64_t nsys0, int64_t nsys1, int64_t row_stride,
                             int64_t sys_stride0, int64_t sys_stride1, const double *a,
                             const double *b, const double *c, const double *shift,
                             const double *d, double *x, int precision, int64_t sys_begin,
                             int64_t sys_end, int32_t *status)
{
    if (!a || !b || !c || !d || !x || n < 1) return ORACLE_EINVAL;
    int64_t nsys = nsys0 * nsys1;
    if (sys_begin < 0 || sys_end > nsys || sys_begin > sys_end) return ORACLE_EINVAL;
    double complex *buf = (double complex *)malloc(5 * (size_t)n * sizeof(double complex));
    if (!buf) return ORACLE_ENOMEM;
    double complex *sa = buf, *sb = buf + n, *sc = buf + 2 * n, *sd = buf + 3 * n, *sx = buf + 4 * n;
    const double complex *dz = (const double complex *)d;
    double complex *xz = (double complex *)x;
    int64_t failed = 0;
    for (int64_t s = sys_begin; s < sys_end; ++s) {
        int64_t s0 = s % nsys0, s1 = s / nsys0;
        int64_t base = s0 * sys_stride0 + s1 * sys_stride1;
        for (int64_t i = 0; i < n; ++i) {
            sa[i] = a[i];
            sb[i] = shift ? b[i] + shift[s] : b[i];
            sc[i] = c[i];
            sd[i] = dz[base + i * row_stride];
        }
        int rc = oracle_thomas_z(n, (const double *)sa, (const double *)sb, (const double *)sc,
                                 (const double *)sd, (double *)sx, precision);
        if (status) status[s] = rc;
        if (rc != ORACLE_OK) { ++failed; continue; }
        for (int64_t i = 0; i < n; ++i) xz[base + i * row_stride] = sx[i];
    }
    free(buf);
    return failed;
}

/*
 * Parallel diagonally dominant (PDD) approximation (Sun 1989; the paper's
 * momentum solver, Sec. 5.1) of one contiguous system, partitions of m rows
 * (the last one shorter when m does not divide n).  Partition k with rows
 * r0..r1 and its own block A_k of A:
 *   A_k xt = d_k,   A_k v = a_{r0} e_first,   A_k w = c_{r1} e_last
 * (v = 0 for the first partition, w = 0 for the last), so that exactly
 *   x_k = xt - v * x_{r0 - 1} - w * x_{r1 + 1}.
 * At the interface between partitions k and k+1 the two unknowns
 * y1 = x_{k,last} and y2 = x_{k+1,first} satisfy, exactly,
 *   y1 + v_k[last] x_{k-1,last} + w_k[last] y2 = xt_k[last]
 *   v_{k+1}[first] y1 + y2 + w_{k+1}[first] x_{k+2,first} = xt_{k+1}[first];
 * PDD drops the two far couplings v_k[last] and w_{k+1}[first] (they decay
 * geometrically with m for a diagonally dominant A), solves the 2 x 2
 * systems independently, and then applies the correction above to every row
 * of every partition with the interface values so found.  With one
 * partition this is the Thomas solve itself.  Each block solve is
 * thomas_f64.  Returns ORACLE_OK, or an error (bad arguments, zero pivot).
 */
int oracle_pdd(int64_t n, const double *a, const double *b, const double *c, const double *d,
               double *x, int64_t m)
{
    if (n < 1 || m < 1 || !a || !b || !c || !d || !x) return ORACLE_EINVAL;
    const int64_t np = (n + m - 1) / m;
    double *xt = (double *)malloc(3 * (size_t)n * sizeof(double));
    double *w2 = (double *)malloc(5 * (size_t)m * sizeof(double));
    double *yl = (double *)malloc(2 * (size_t)np * sizeof(double));   /* x_{k,last}, x_{k,first} */
    if (!xt || !w2 || !yl) { free(xt); free(w2); free(yl); return ORACLE_ENOMEM; }
    double *v = xt + n, *w = xt + 2 * n;
    double *cp = w2, *dp = w2 + m, *rhs = w2 + 2 * m, *sb = w2 + 3 * m, *sa = w2 + 4 * m;
    int rc = ORACLE_OK;
    for (int64_t k = 0; k < np && rc == ORACLE_OK; ++k) {
        const int64_t r0 = k * m, len = (r0 + m <= n) ? m : n - r0;
        /* the block A_k: sub-diagonal without its first entry, super-diagonal
         * without its last (those couple to the neighbours) */
        for (int64_t i = 0; i < len; ++i) { sa[i] = (i > 0) ? a[r0 + i] : 0.0; sb[i] = b[r0 + i]; }
        double *sc = rhs;   /* reuse: super-diagonal of the block */
        for (int64_t i = 0; i < len; ++i) sc[i] = (i < len - 1) ? c[r0 + i] : 0.0;
        rc = thomas_f64(len, sa, sb, sc, d + r0, xt + r0, cp, dp);
        if (rc != ORACLE_OK) break;
        double *e = (double *)malloc((size_t)len * sizeof(double));
        if (!e) { rc = ORACLE_ENOMEM; break; }
        for (int64_t i = 0; i < len; ++i) e[i] = 0.0;
        if (k > 0) e[0] = a[r0];
        rc = thomas_f64(len, sa, sb, sc, e, v + r0, cp, dp);
        for (int64_t i = 0; i < len; ++i) e[i] = 0.0;
        if (rc == ORACLE_OK && k < np - 1) {
            e[len - 1] = c[r0 + len - 1];
            rc = thomas_f64(len, sa, sb, sc, e, w + r0, cp, dp);
        } else if (rc == ORACLE_OK) {
            for (int64_t i = 0; i < len; ++i) w[r0 + i] = 0.0;
        }
        free(e);
    }
    if (rc == ORACLE_OK) {
        /* interface k | k+1: y1 = x_{k,last}, y2 = x_{k+1,first} */
        for (int64_t k = 0; k + 1 < np; ++k) {
            const int64_t last = (k + 1) * m - 1, first = last + 1;
            const double det = 1.0 - w[last] * v[first];
            if (det == 0.0 || !isfinite(det)) { rc = ORACLE_ESINGULAR; break; }
            yl[2 * k] = (xt[last] - w[last] * xt[first]) / det;
            yl[2 * (k + 1) + 1] = (xt[first] - v[first] * xt[last]) / det;
        }
    }
    if (rc == ORACLE_OK) {
        for (int64_t k = 0; k < np; ++k) {
            const int64_t r0 = k * m, len = (r0 + m <= n) ? m : n - r0;
            const double left = (k > 0) ? yl[2 * (k - 1)] : 0.0;           /* x_{k-1,last} */
            const double right = (k < np - 1) ? yl[2 * (k + 1) + 1] : 0.0;  /* x_{k+1,first} */
            for (int64_t i = 0; i < len; ++i)
                x[r0 + i] = xt[r0 + i] - v[r0 + i] * left - w[r0 + i] * right;
        }
    }
    free(xt);
    free(w2);
    free(yl);
    return rc;
}

/* y = A x for one contiguous system (FP64, no FMA): the residual check's
 * matrix-vector product.  a[0] and c[n-1] are not read. */
void oracle_matvec(int64_t n, const double *a, const double *b, const double *c,
                   const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = b[i] * x[i];
        if (i > 0) v += a[i] * x[i - 1];
        if (i < n - 1) v += c[i] * x[i + 1];
        y[i] = v;
    }
}
