/*
 * CPU oracle for the batched parallel-prefix operations -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * call this library.  It shares no code with the GPU library: it is the plain
 * mathematical definition of each operation, written out in double precision
 * (inputs given in single precision or int32 are promoted exactly), with no
 * blocking, fusion or reordering beyond what the definition states.
 *
 *   oracle_dft       complex DFT by its O(N^2) definition (Sec. III, "Fast
 *                    Fourier Transform": the complex FFT the Stockham kernels
 *                    compute; Sec. VI-C gives the 5 N log2 N flop convention).
 *   oracle_dft_bins  selected outputs of that DFT, each by the definition.
 *   oracle_scan_u32  inclusive sum scan, integer: each output is the sum of
 *                    all inputs up to and including itself (Sec. III, "Scan
 *                    Operator"); arithmetic modulo 2^32.
 *   oracle_scan_f64  the same scan in double precision.
 *   oracle_scan_excl_u32, oracle_scan_excl_f64
 *                    the exclusive scan: each output is the sum of the
 *                    inputs strictly before it (0 for the first).
 *   oracle_thomas    the solution of the tridiagonal system
 *                    a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i (Sec. III,
 *                    "Tridiagonal system solvers"), x_{-1} = x_N = 0, by
 *                    Gaussian elimination without pivoting specialised to the
 *                    tridiagonal band (the Thomas algorithm).
 *   oracle_tridiag_residual
 *                    ||A x - d||_2 / ||d||_2 per system, in double precision.
 *
 * Every entry point takes `batch` independent problems of size `n` stored
 * row-major ([batch][n]); they are spread over `nthreads` POSIX threads
 * (0 = all online CPUs), one contiguous range of problems per thread.
 * Return value: 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef void (*problem_fn)(void *ctx, int64_t first, int64_t last);

typedef struct {
    problem_fn fn;
    void *ctx;
    int64_t first, last;
} range_job;

static void *range_thread(void *arg)
{
    range_job *j = (range_job *)arg;
    j->fn(j->ctx, j->first, j->last);
    return NULL;
}

/* Run fn over problems [0, batch) split into nthreads contiguous ranges. */
static int run_ranges(problem_fn fn, void *ctx, int64_t batch, int nthreads)
{
    if (nthreads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        nthreads = c > 0 ? (int)c : 1;
    }
    if ((int64_t)nthreads > batch)
        nthreads = (int)(batch > 0 ? batch : 1);
    if (nthreads == 1) {
        fn(ctx, 0, batch);
        return 0;
    }
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    range_job *jobs = (range_job *)calloc((size_t)nthreads, sizeof(range_job));
    int *started = (int *)calloc((size_t)nthreads, sizeof(int));
    if (!th || !jobs || !started) {
        free(th); free(jobs); free(started);
        return -2;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].first = batch * t / nthreads;
        jobs[t].last = batch * (t + 1) / nthreads;
        started[t] = pthread_create(&th[t], NULL, range_thread, &jobs[t]) == 0;
        if (!started[t])
            fn(ctx, jobs[t].first, jobs[t].last); /* run inline instead */
    }
    for (int t = 0; t < nthreads; ++t)
        if (started[t])
            pthread_join(th[t], NULL);
    free(th); free(jobs); free(started);
    return 0;
}

/* ------------------------------------------------------------------ DFT -- */

typedef struct {
    const double *x; /* interleaved (re, im), [batch][n][2] */
    double *X;
    const double *wre, *wim; /* w[m] = exp(sign * 2 pi i m / n), m < n */
    int64_t n;
} dft_ctx;

static void dft_range(void *vctx, int64_t first, int64_t last)
{
    dft_ctx *c = (dft_ctx *)vctx;
    const int64_t n = c->n;
    for (int64_t b = first; b < last; ++b) {
        const double *x = c->x + 2 * n * b;
        double *X = c->X + 2 * n * b;
        for (int64_t k = 0; k < n; ++k) {
            double sre = 0.0, sim = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                /* exact reduction of the exponent j*k modulo n */
                const int64_t m = (j * k) % n;
                const double xr = x[2 * j], xi = x[2 * j + 1];
                sre += xr * c->wre[m] - xi * c->wim[m];
                sim += xr * c->wim[m] + xi * c->wre[m];
            }
            X[2 * k] = sre;
            X[2 * k + 1] = sim;
        }
    }
}

/*
 * X[b][k] = sum_{j<n} x[b][j] * exp(sign * 2 pi i j k / n), sign = -1 for the
 * forward transform and +1 for the (unnormalised) inverse.  Any n >= 1.
 */
int oracle_dft(const double *x, double *X, int64_t n, int64_t batch, int sign,
               int nthreads)
{
    if (!x || !X || n < 1 || batch < 0 || (sign != -1 && sign != 1))
        return -1;
    double *wre = (double *)malloc(sizeof(double) * (size_t)n);
    double *wim = (double *)malloc(sizeof(double) * (size_t)n);
    if (!wre || !wim) {
        free(wre); free(wim);
        return -2;
    }
    for (int64_t m = 0; m < n; ++m) {
        const double ang = 2.0 * M_PI * (double)m / (double)n;
        wre[m] = cos(ang);
        wim[m] = (double)sign * sin(ang);
    }
    dft_ctx ctx = {x, X, wre, wim, n};
    int rc = run_ranges(dft_range, &ctx, batch, nthreads);
    free(wre); free(wim);
    return rc;
}

/*
 * Selected bins of the same DFT: X[b][i] = sum_{j<n} x[b][j] * exp(sign * 2 pi
 * i j ks[i] / n) for i < nk, each bin by the definition (O(n) per bin), for
 * sizes whose full O(n^2) transform is too slow to check every output.
 */
typedef struct {
    const double *x;
    double *X; /* [batch][nk][2] */
    const double *wre, *wim;
    const int64_t *ks;
    int64_t n, nk;
} bins_ctx;

static void bins_range(void *vctx, int64_t first, int64_t last)
{
    bins_ctx *c = (bins_ctx *)vctx;
    const int64_t n = c->n;
    for (int64_t job = first; job < last; ++job) {
        const int64_t b = job / c->nk, i = job % c->nk;
        const int64_t k = c->ks[i];
        const double *x = c->x + 2 * n * b;
        double sre = 0.0, sim = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t m = (j * k) % n;
            const double xr = x[2 * j], xi = x[2 * j + 1];
            sre += xr * c->wre[m] - xi * c->wim[m];
            sim += xr * c->wim[m] + xi * c->wre[m];
        }
        c->X[2 * job] = sre;
        c->X[2 * job + 1] = sim;
    }
}

int oracle_dft_bins(const double *x, double *X, int64_t n, int64_t batch, const int64_t *ks,
                    int64_t nk, int sign, int nthreads)
{
    if (!x || !X || !ks || n < 1 || batch < 0 || nk < 0 || (sign != -1 && sign != 1))
        return -1;
    for (int64_t i = 0; i < nk; ++i)
        if (ks[i] < 0 || ks[i] >= n)
            return -1;
    double *wre = (double *)malloc(sizeof(double) * (size_t)n);
    double *wim = (double *)malloc(sizeof(double) * (size_t)n);
    if (!wre || !wim) {
        free(wre); free(wim);
        return -2;
    }
    for (int64_t m = 0; m < n; ++m) {
        const double ang = 2.0 * M_PI * (double)m / (double)n;
        wre[m] = cos(ang);
        wim[m] = (double)sign * sin(ang);
    }
    bins_ctx ctx = {x, X, wre, wim, ks, n, nk};
    int rc = run_ranges(bins_range, &ctx, batch * nk, nthreads);
    free(wre); free(wim);
    return rc;
}

/* ----------------------------------------------------------------- scan -- */

typedef struct {
    const void *x;
    void *y;
    int64_t n;
} scan_ctx;

static void scan_u32_range(void *vctx, int64_t first, int64_t last)
{
    scan_ctx *c = (scan_ctx *)vctx;
    const uint32_t *x = (const uint32_t *)c->x;
    uint32_t *y = (uint32_t *)c->y;
    for (int64_t b = first; b < last; ++b) {
        uint32_t acc = 0u;
        for (int64_t i = 0; i < c->n; ++i) {
            acc += x[b * c->n + i]; /* unsigned: wraps modulo 2^32 */
            y[b * c->n + i] = acc;
        }
    }
}

static void scan_f64_range(void *vctx, int64_t first, int64_t last)
{
    scan_ctx *c = (scan_ctx *)vctx;
    const double *x = (const double *)c->x;
    double *y = (double *)c->y;
    for (int64_t b = first; b < last; ++b) {
        double acc = 0.0;
        for (int64_t i = 0; i < c->n; ++i) {
            acc += x[b * c->n + i];
            y[b * c->n + i] = acc;
        }
    }
}

/* y[b][i] = sum_{j<=i} x[b][j]  (mod 2^32; int32 inputs viewed as uint32). */
int oracle_scan_u32(const uint32_t *x, uint32_t *y, int64_t n, int64_t batch,
                    int nthreads)
{
    if (!x || !y || n < 1 || batch < 0)
        return -1;
    scan_ctx ctx = {x, y, n};
    return run_ranges(scan_u32_range, &ctx, batch, nthreads);
}

/* y[b][i] = sum_{j<=i} x[b][j] in double precision, summed left to right. */
int oracle_scan_f64(const double *x, double *y, int64_t n, int64_t batch,
                    int nthreads)
{
    if (!x || !y || n < 1 || batch < 0)
        return -1;
    scan_ctx ctx = {x, y, n};
    return run_ranges(scan_f64_range, &ctx, batch, nthreads);
}

/* Exclusive form: every output is the sum of the inputs strictly before it,
 * so the first output of each problem is 0 (the scan operator of Sec. III
 * with the element itself left out). */
static void scan_excl_u32_range(void *vctx, int64_t first, int64_t last)
{
    scan_ctx *c = (scan_ctx *)vctx;
    const uint32_t *x = (const uint32_t *)c->x;
    uint32_t *y = (uint32_t *)c->y;
    for (int64_t b = first; b < last; ++b) {
        uint32_t before = 0u;
        for (int64_t i = 0; i < c->n; ++i) {
            const uint32_t xi = x[b * c->n + i]; /* read first: y may be x */
            y[b * c->n + i] = before;
            before += xi;
        }
    }
}

static void scan_excl_f64_range(void *vctx, int64_t first, int64_t last)
{
    scan_ctx *c = (scan_ctx *)vctx;
    const double *x = (const double *)c->x;
    double *y = (double *)c->y;
    for (int64_t b = first; b < last; ++b) {
        double before = 0.0;
        for (int64_t i = 0; i < c->n; ++i) {
            const double xi = x[b * c->n + i];
            y[b * c->n + i] = before;
            before += xi;
        }
    }
}

/* y[b][i] = sum_{j<i} x[b][j]  (mod 2^32), y[b][0] = 0. */
int oracle_scan_excl_u32(const uint32_t *x, uint32_t *y, int64_t n, int64_t batch,
                         int nthreads)
{
    if (!x || !y || n < 1 || batch < 0)
        return -1;
    scan_ctx ctx = {x, y, n};
    return run_ranges(scan_excl_u32_range, &ctx, batch, nthreads);
}

/* y[b][i] = sum_{j<i} x[b][j] in double precision, summed left to right. */
int oracle_scan_excl_f64(const double *x, double *y, int64_t n, int64_t batch,
                         int nthreads)
{
    if (!x || !y || n < 1 || batch < 0)
        return -1;
    scan_ctx ctx = {x, y, n};
    return run_ranges(scan_excl_f64_range, &ctx, batch, nthreads);
}

/* -------------------------------------------------------- tridiagonal -- */

typedef struct {
    const double *a, *b, *c, *d;
    double *x;
    double *rel;
    int64_t n;
    int status; /* set nonzero if a pivot is exactly zero */
} tri_ctx;

static void thomas_range(void *vctx, int64_t first, int64_t last)
{
    tri_ctx *t = (tri_ctx *)vctx;
    const int64_t n = t->n;
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    double *dp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cp || !dp) {
        free(cp); free(dp);
        t->status = -2;
        return;
    }
    for (int64_t s = first; s < last; ++s) {
        const double *a = t->a + s * n, *b = t->b + s * n;
        const double *c = t->c + s * n, *d = t->d + s * n;
        double *x = t->x + s * n;
        /* a[0] and c[n-1] multiply the absent unknowns x_{-1}, x_n: unused. */
        for (int64_t i = 0; i < n; ++i) {
            const double ai = (i == 0) ? 0.0 : a[i];
            const double ci = (i == n - 1) ? 0.0 : c[i];
            const double m = b[i] - ai * (i == 0 ? 0.0 : cp[i - 1]);
            if (m == 0.0)
                t->status = -3;
            cp[i] = ci / m;
            dp[i] = (d[i] - ai * (i == 0 ? 0.0 : dp[i - 1])) / m;
        }
        x[n - 1] = dp[n - 1];
        for (int64_t i = n - 2; i >= 0; --i)
            x[i] = dp[i] - cp[i] * x[i + 1];
    }
    free(cp); free(dp);
}

/*
 * Solve a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i < n, for each system.
 * a[.][0] and c[.][n-1] are never read as coefficients.  Returns -3 if a zero
 * pivot was met (the inputs of the diagonally dominant recipe never do).
 */
int oracle_thomas(const double *a, const double *b, const double *c,
                  const double *d, double *x, int64_t n, int64_t batch,
                  int nthreads)
{
    if (!a || !b || !c || !d || !x || n < 1 || batch < 0)
        return -1;
    tri_ctx ctx = {a, b, c, d, x, NULL, n, 0};
    int rc = run_ranges(thomas_range, &ctx, batch, nthreads);
    return rc ? rc : ctx.status;
}

static void residual_range(void *vctx, int64_t first, int64_t last)
{
    tri_ctx *t = (tri_ctx *)vctx;
    const int64_t n = t->n;
    for (int64_t s = first; s < last; ++s) {
        const double *a = t->a + s * n, *b = t->b + s * n;
        const double *c = t->c + s * n, *d = t->d + s * n;
        const double *x = t->x + s * n;
        double rr = 0.0, dd = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double r = b[i] * x[i] - d[i];
            if (i > 0)
                r += a[i] * x[i - 1];
            if (i < n - 1)
                r += c[i] * x[i + 1];
            rr += r * r;
            dd += d[i] * d[i];
        }
        t->rel[s] = dd > 0.0 ? sqrt(rr) / sqrt(dd) : sqrt(rr);
    }
}

/* rel[s] = ||A_s x_s - d_s||_2 / ||d_s||_2 (absolute norm if d_s = 0). */
int oracle_tridiag_residual(const double *a, const double *b, const double *c,
                            const double *d, const double *x, double *rel,
                            int64_t n, int64_t batch, int nthreads)
{
    if (!a || !b || !c || !d || !x || !rel || n < 1 || batch < 0)
        return -1;
    tri_ctx ctx = {a, b, c, d, (double *)x, rel, n, 0};
    return run_ranges(residual_range, &ctx, batch, nthreads);
}
