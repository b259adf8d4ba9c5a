/*
 * ppx.h -- C ABI of libppx.so: batched power-of-two parallel-prefix
 * operations (complex FFT, inclusive scan, tridiagonal solve) for AMD MI355X
 * (gfx950), and the tuners that choose their launch parameters.
 *
 * Source of the operations: arXiv:2310.16214, Sec. III (definitions of the
 * tridiagonal system, the scan operator and the Stockham complex FFT), Sec.
 * IV-A (the tunable tuple (S,P,L), radix r, and batched execution of G
 * problems of size N = r^n per invocation), Sec. IV-B and Table
 * "parameters-TL" (the performance-parameter space and the Bayesian search),
 * Sec. VI (data resident on the GPU; the Phi metric).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Problems are stored row-major, [batch][n], contiguous, problem stride n.
 *   Device pointers must be 16-byte aligned.  The caller owns every buffer;
 *   the compute entry points allocate nothing.
 * - n must be a power of two in [PPX_MIN_N, PPX_MAX_N]; batch >= 1.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Compute calls are asynchronous and stream-ordered.
 * - `cfg` may be NULL: the library then uses the configuration recorded by
 *   tune() for (op, dtype, n) if there is one, else the analytical model's
 *   choice.  An explicit cfg is validated (ppx_config_valid) and rejected
 *   with PPX_ECONFIG if it does not describe a valid launch.
 * - Every call returns PPX_OK (0) or a negative PPX_E* code; a message is
 *   then available from ppx_last_error() (thread-local).  Argument checks run
 *   before any HIP runtime call, so they need no GPU.
 */
#ifndef PPX_H
#define PPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define PPX_OK 0
#define PPX_EINVAL (-1)   /* null/misaligned pointer, bad n, batch, dtype, op */
#define PPX_ECONFIG (-2)  /* explicit configuration is not a valid launch */
#define PPX_EDEVICE (-3)  /* current device is not gfx950 / no device */
#define PPX_EHIP (-4)     /* a HIP runtime call or kernel launch failed */
#define PPX_ENOMEM (-5)   /* allocation failed (tune, server, graph only) */
#define PPX_ETIMEOUT (-6) /* a timed candidate exceeded its deadline */

/* ---- data types ---- */
#define PPX_I32 0
#define PPX_F32 1
#define PPX_F64 2
#define PPX_C64 3 /* interleaved complex float (re, im) */

/* ---- operations ---- */
#define PPX_OP_FFT 0
#define PPX_OP_SCAN 1
#define PPX_OP_TRIDIAG 2

/* ---- algorithm selectors (ppx_config.algo) ---- */
#define PPX_FFT_LDS 0       /* exchange complex values through LDS */
#define PPX_FFT_LDS_SPLIT 1 /* real parts, then imaginary parts, through a
                               half-size LDS buffer (Sec. V-C) */
#define PPX_FFT_LDS_PIPE 2  /* PPX_FFT_LDS in persistent workgroups (as many as
                               are resident) that load the next group of
                               problems into registers while transforming the
                               current one; radix = P = 8 or 16 only */
#define PPX_FFT_LDS_SPLIT_PIPE 3 /* PPX_FFT_LDS_SPLIT, persistent as above */
#define PPX_SCAN_KS 0       /* Kogge-Stone lane network (DPP row shifts) */
#define PPX_SCAN_LF 1       /* Ladner-Fischer lane network (swizzle bcasts) */
#define PPX_SCAN_KS_PIPE 2  /* PPX_SCAN_KS in persistent workgroups (as many as
                               are resident) that load the next group of
                               problems while scanning the current one */
#define PPX_SCAN_LF_PIPE 3  /* PPX_SCAN_LF, persistent as above */
#define PPX_TRI_CR 0        /* cyclic reduction (Sec. III), LDS exchange */
#define PPX_TRI_PCR 1       /* parallel cyclic reduction (Sec. III), LDS exchange */
#define PPX_TRI_CR_PCR 2    /* CR -> PCR hybrid inside a wave (S = 0): the CR
                               levels inside each lane reduce its P equations
                               to one, PCR solves the n / P remaining ones
                               across the lanes, back substitution inside the
                               lane recovers the rest; n / P <= 64, P <= 16 */
#define PPX_TRI_CR_SHFL 3   /* CR inside a wave: registers + lane shuffles, no
                               LDS (S = 0); valid when n / P <= 64, P <= 16 */
#define PPX_TRI_PCR_SHFL 4  /* PCR inside a wave (S = 0); n / P <= 64, P <= 16 */
#define PPX_TRI_PCR_REG 5   /* PCR inside a wave, the cross-lane exchange through
                               a per-wave LDS buffer of 3 * 64 * min(P, 4)
                               values (16-byte accesses) instead of shuffles;
                               S = 0, n / P <= 64, P <= 16 */
#define PPX_TRI_WM 6        /* Wang & Mou divide and conquer inside a wave
                               (Sec. III): blocks of equations merge in pairs,
                               each equation kept solved in terms of its
                               block's two outer unknowns; radix P (a lane's P
                               equations form the first node), then radix 2
                               across lanes by broadcasts; S = 0, n / P <= 64,
                               P <= 16 */
#define PPX_TRI_LF 7        /* Ladner-Fischer solver inside a wave (Sec. III):
                               a prefix scan (Ladner-Fischer circuit) over
                               elements of two equations, the first and last
                               of a block, then one over the back-substitution
                               maps; S = 0, n / P <= 64, P <= 16 */
#define PPX_TRI_PIPE 8      /* flag, OR-ed onto an in-wave variant (PPX_TRI_CR_PCR,
                               _CR_SHFL, _PCR_SHFL, _PCR_REG, _WM or _LF):
                               persistent workgroups (as many as are
                               resident) that load the next group of systems
                               while solving the current one */

/* ---- tuning methods ---- */
#define PPX_TUNE_EXHAUSTIVE 0 /* time every valid configuration (Sec. VI) */
#define PPX_TUNE_ANALYTICAL 1 /* occupancy guideline, no timing (Sec. IV-A) */
#define PPX_TUNE_LEARNED 2    /* Bayesian optimisation, GP + EI (Sec. IV-B) */

#define PPX_MIN_N 16
#define PPX_MAX_N 16384

/*
 * Launch parameters of one batched call (Sec. IV-A's (S,P,L) and radix r,
 * plus G_b, the problems solved by one workgroup).
 *   radix               r: FFT butterfly radix in {2,4,8,16}; 2 for scan and
 *                       tridiagonal.  When log2(n) is not a multiple of
 *                       log2(r) the first FFT stage uses the lower radix
 *                       2^(log2 n mod log2 r).
 *   elems_per_thread    P = n * G_b / L; 0 means "derive from L and G_b".
 *   threads_per_block   L in {64,128,256,512,1024}.
 *   problems_per_block  G_b in {1,2,4,...}; G_b * n = P * L.
 *   lds_elems           S, elements held in LDS per workgroup; 0 on input
 *                       means "derive"; ppx_resolve_config reports the value.
 *   algo                PPX_FFT_*, PPX_SCAN_* or PPX_TRI_*.
 */
typedef struct ppx_config {
    int32_t radix;
    int32_t elems_per_thread;
    int32_t threads_per_block;
    int32_t problems_per_block;
    int32_t lds_elems;
    int32_t algo;
} ppx_config;

/*
 * fft_batched -- Sec. III (Stockham complex FFT), Sec. IV-A (batched).
 * For every problem b < batch:
 *   out[b][k] = sum_{j<n} in[b][j] * exp(direction * 2*pi*i * j*k / n)
 * direction = -1 (forward) or +1 (inverse); neither is normalised.  Output is
 * in natural order.  in/out: device pointers to batch*n interleaved complex
 * floats (PPX_C64).  in == out (in place) is allowed; partial overlap is not.
 * For PPX_MAX_N < n <= PPX_MAX_N_LARGE see fft_batched_large (cfg must then
 * be NULL).
 */
int fft_batched(const void *in, void *out, int64_t n, int64_t batch,
                int direction, const ppx_config *cfg, void *stream);

/*
 * Large-N FFT (PPX_MAX_N < n <= PPX_MAX_N_LARGE) -- the multi-kernel case of
 * Sec. IV-A: n = n1 * n2 is transformed by two launches of column FFTs (pass
 * A over the n2 dimension of the input viewed as n2 rows of n1 columns, with
 * the twiddles w_n^{j1 k2}, writing the transposed intermediate to `out`;
 * pass B over the n1 dimension, in place in `out`).  A plan fixes the split
 * and each pass's radix (= values per thread):
 *   log2_n1    log2 n1; both passes need a column length in the range their
 *              radix and tile support (radix 16 from 2^6, radix 8 from
 *              2^5; beyond 2^10 only narrow tiles, up to 2^12 in pass A
 *              and 2^13 in pass B)
 *   radix_a    radix of pass A (column length n2 = n / n1)
 *   radix_b    radix of pass B (column length n1)
 *   tile_a     columns per workgroup of pass A
 *   tile_b     columns per workgroup of pass B: 16, 32 or 64 for columns of
 *              up to 1024 values, 2, 4 or 8 for longer ones
 * A pass's workgroup transforms tile adjacent columns of length len with
 * tile * len / radix threads (64..1024) and tile * (len + 1) complex values
 * of LDS (<= 160 KiB, with 2056 more for pass A's twiddle tables, and the
 * stage twiddle bases where a tile leaves room for one workgroup per CU and
 * runs persistent); the tile must divide the pass's column count (n1 for
 * pass A, n2 for pass B).  Tuning the plan (tune_fft_large) is the
 * interdependent per-kernel search of the paper's learned tuner.
 */
#define PPX_MAX_N_LARGE 8388608
typedef struct ppx_fft_plan {
    int32_t log2_n1;
    int32_t radix_a;
    int32_t radix_b;
    int32_t tile_a;
    int32_t tile_b;
} ppx_fft_plan;

/*
 * fft_batched_large -- same transform and conventions as fft_batched, for
 * PPX_MAX_N < n <= PPX_MAX_N_LARGE.  in and out must not overlap at all (out
 * holds the intermediate between the passes).  plan == NULL: the plan
 * tune_fft_large recorded for n, else ppx_default_fft_plan.  Errors:
 * PPX_EINVAL (pointers, n, batch, direction, overlap), PPX_ECONFIG (plan).
 * fft_batched with such an n and cfg == NULL forwards here.
 */
int fft_batched_large(const void *in, void *out, int64_t n, int64_t batch, int direction,
                      const ppx_fft_plan *plan, void *stream);

/* PPX_OK if plan is valid for n, else PPX_ECONFIG (reason in ppx_last_error()). */
int ppx_fft_plan_valid(int64_t n, const ppx_fft_plan *plan);

/*
 * Every valid plan for n, ordered by log2_n1, radix_a, radix_b, tile_a, tile_b:
 * writes min(count, cap) plans to out (out may be NULL when cap == 0) and
 * returns the count, or a negative PPX_E* code.
 */
int ppx_enumerate_fft_plans(int64_t n, ppx_fft_plan *out, int cap);

/*
 * The untuned plan: the most even valid split (n1 <= n2 on a tie) and, in
 * each pass, the widest tile of at most 16 columns, with radix 8 where both
 * radices allow it.  The analytical plan (tune_fft_large with
 * PPX_TUNE_ANALYTICAL) is the gfx950 occupancy guideline applied per pass.
 */
int ppx_default_fft_plan(int64_t n, ppx_fft_plan *out);

/*
 * tune_fft_large -- tune() for the large-N FFT: the candidates are the valid
 * plans for n, timed as whole two-pass calls (median of 100 after warm-ups,
 * rotating buffer sets as in tune()).  EXHAUSTIVE times every plan, LEARNED
 * runs the Bayesian search over the plan features (log2 of n1, both radices
 * and both tile widths), ANALYTICAL applies the occupancy guideline to each
 * pass's kernels separately over its (radix, tile) choices and takes the
 * most even split.
 * The winner is recorded for fft_batched_large(plan == NULL).
 */
int tune_fft_large(int64_t n, int64_t batch, int method, int max_evals, ppx_fft_plan *best,
                   double *best_us, int *evals_used);

/*
 * scan_batched -- Sec. III ("Scan Operator"): inclusive sum scan,
 *   out[b][i] = sum_{j<=i} in[b][j]
 * in, out: device arrays [batch][n], 16-byte aligned, of dtype PPX_I32 (wraps
 * modulo 2^32, bit-exact), PPX_F32 or PPX_F64 (float64: at most 16 elements
 * per thread).  in == out is allowed; partial overlap is not.
 */
int scan_batched(const void *in, void *out, int64_t n, int64_t batch,
                 int dtype, const ppx_config *cfg, void *stream);

/*
 * scan_exclusive_batched -- the exclusive form of the scan operator of
 * Sec. III (the prescan): out[b][i] = sum_{j<i} in[b][j], out[b][0] = 0.
 * Arguments, dtypes, aliasing and the configuration space as for
 * scan_batched; cfg == NULL takes the configuration scan_batched would use
 * (the two kernels differ only in the thread-serial step).
 */
int scan_exclusive_batched(const void *in, void *out, int64_t n, int64_t batch,
                           int dtype, const ppx_config *cfg, void *stream);

/*
 * tridiag_batched -- Sec. III (tridiagonal system solvers, CR and PCR):
 * solves a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i < n, for each system.
 * a, b, c, d, x: device arrays [batch][n] of dtype PPX_F32 or PPX_F64 (four
 * separate coefficient arrays).  a[.][0] and c[.][n-1] multiply absent
 * unknowns: their stored values, even NaN, do not affect x.  x may equal d
 * (the solve then overwrites the right-hand side); no other aliasing.
 * No pivoting: systems are assumed diagonally dominant.  cfg->algo picks CR
 * or PCR and the exchange (LDS, or lane shuffles when a system fits a wave:
 * the paper's "shuffle" option).  Every variant keeps each equation scaled to
 * unit diagonal (one reciprocal per elimination, a refined hardware estimate
 * rather than IEEE division); the solution is that of the unscaled system.
 */
int tridiag_batched(const void *a, const void *b, const void *c, const void *d,
                    void *x, int64_t n, int64_t batch, int dtype,
                    const ppx_config *cfg, void *stream);

/*
 * tune -- Sec. IV (analytical and learned tuning) and Sec. VI (exhaustive
 * search as the reference).  Chooses a configuration for (op, dtype, n) at
 * the given batch on the current device and records it in the tune cache,
 * where later calls with cfg == NULL find it.
 *   method     PPX_TUNE_EXHAUSTIVE | PPX_TUNE_ANALYTICAL | PPX_TUNE_LEARNED
 *   max_evals  cap on timed candidates (<= 0: no cap); ignored for
 *              ANALYTICAL, which times nothing.
 *   best       receives the chosen configuration (required).
 *   best_us    receives its median time in microseconds (NULL allowed; for
 *              ANALYTICAL the chosen config is timed once for reporting).
 *   evals_used receives the number of timed candidates (NULL allowed).
 * Synchronous.  Allocates and frees its own scratch buffers (inputs are
 * seeded synthetic data).  For op == PPX_OP_FFT, dtype must be PPX_C64.
 * The cache file is $PPX_TUNE_CACHE if set, else none (in-memory only).
 */
int tune(int op, int dtype, int64_t n, int64_t batch, int method, int max_evals,
         ppx_config *best, double *best_us, int *evals_used);

/*
 * One job of a mixed launch: a whole batched call of any operation.
 *   op, dtype, n, batch   as in the single calls
 *   direction             FFT only: -1 forward, +1 inverse
 *   algo                  tridiagonal: the solver family, PPX_TRI_CR,
 *                         PPX_TRI_PCR, PPX_TRI_WM or PPX_TRI_LF; scan:
 *                         PPX_JOB_SCAN_INCLUSIVE or PPX_JOB_SCAN_EXCLUSIVE
 *                         (dtype PPX_I32, PPX_F32 or PPX_F64)
 *   in                    FFT / scan input; tridiagonal: a
 *   b, c, d               tridiagonal only (NULL otherwise)
 *   out                   FFT / scan output; tridiagonal: x
 * Device pointers, 16-byte aligned, caller-owned; aliasing as in the single
 * calls.  Tridiagonal systems solved through LDS (n > 1024) must fit 128 KiB
 * (float32 CR: n <= 8192; PCR or float64: n <= 4096; float64 PCR: n <= 2048).
 */
#define PPX_JOB_SCAN_INCLUSIVE 0
#define PPX_JOB_SCAN_EXCLUSIVE 1
typedef struct ppx_job {
    int32_t op;
    int32_t dtype;
    int32_t direction;
    int32_t algo;
    int64_t n;
    int64_t batch;
    const void *in;
    const void *b;
    const void *c;
    const void *d;
    void *out;
} ppx_job;

/*
 * launch_mixed -- Sec. IV-A's batched invocation extended to a batch of
 * uneven jobs (different operations, sizes and batch counts) in one launch.
 * Each job is cut into tiles of the shape its single call uses with
 * cfg == NULL (the tuned configuration, else the analytical one;
 * tridiagonal: of the job's family): the same radix, values per thread and
 * solver, so each job's output equals that single call's and does not
 * depend on what else shares the launch.  The tiles run in one kernel per
 * family of tile shapes (FFT, scan and tridiagonal by block size and
 * register demand).  A launch with at most PPX_MIXED_ARG_JOBS jobs in every
 * family passes the job records in the kernel arguments, one workgroup per
 * tile: one kernel launch per family and nothing else.  A larger launch
 * copies its tables to the device (one of 4 ring slots), expands the tile
 * lists and runs persistent kernels that claim tiles from per-family
 * counters.  Asynchronous and stream-ordered; allocates nothing after a
 * device's first mixed launch, which creates the ring slots.  At most 16384
 * jobs and 2^20 tiles per launch (PPX_EINVAL beyond).
 */
int launch_mixed(const ppx_job *jobs, int njobs, void *stream);
/* A job of at least this many elements (n * batch) whose configuration with
 * cfg == NULL is a persistent variant runs, inside launch_mixed, as that
 * single call, after the tiled jobs: it fills the GPU by itself, and the
 * persistent kernel prefetches its next group while computing the current
 * one, which a tile of the shared loop cannot.  Still a pure function of the
 * job, so its output is the same alone or in any mix. */
#define PPX_MIXED_DIRECT_ELEMS (1LL << 22)

/*
 * launch_mixed_noalloc -- launch_mixed for callers that cannot allocate
 * device or pinned memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same jobs, tiles, kernels and results
 * as launch_mixed (bit-identical outputs); the launch tables live in a
 * static device array of about 1 MiB that the library holds on each device
 * until the process ends.  At most PPX_NOALLOC_MAX_JOBS jobs and
 * PPX_NOALLOC_MAX_TILES tiles per call (PPX_EINVAL beyond; the tile count of
 * a job is its batch over ppx_mixed_tile_config's problems per tile).  The
 * caller passes the inputs and outputs.  The first call on a device sets it
 * up (device state, occupancy queries, the array's address) without
 * allocating; later calls only plan on the host and enqueue, on `stream`,
 * what launch_mixed does: the argument kernels for a launch with few jobs
 * per family (the array unused), else a few table copy kernels, the
 * tile-list expansion and the persistent family kernels.
 * Every call on a device shares that device's array, so calls whose work
 * overlaps on one device (different streams, or host threads) race and must
 * be ordered by the caller.  Host-side planning touches no heap for shapes
 * whose configuration is in the tune cache or was resolved before (the
 * analytical choice is memoised on its first use); a caller under graph
 * capture can resolve its shapes once beforehand (ppx_mixed_tile_config).
 * Asynchronous and stream-ordered.
 */
#define PPX_NOALLOC_MAX_JOBS 256
#define PPX_NOALLOC_MAX_TILES 262144
int launch_mixed_noalloc(const ppx_job *jobs, int njobs, void *stream);

/*
 * ppx_mixed_tile_config -- how launch_mixed cuts *job: returns the problems
 * per tile (> 0) of the job in a launch of its own (the configuration's
 * problems per workgroup where its workgroup size is within the tile
 * kernel's limit; a launch runs each family at the largest workgroup size of
 * its jobs, so a job may get more problems per tile there, and a launch too
 * small to fill the GPU fewer) or a negative PPX_E* code, and writes to *cfg
 * (if not NULL) the single-call configuration whose arithmetic the tiles
 * follow:
 * the configuration of the job's call with cfg == NULL, with the persistent
 * flag cleared (a launch strategy, not arithmetic); for a job that runs as
 * its own call (PPX_MIXED_DIRECT_ELEMS), that configuration unchanged and its
 * problems per workgroup; for an FFT whose tuned
 * shape is not radix = P in {8, 16} (or 4 with n <= 1024), the radix = P
 * shape used instead.  A single call with that configuration gives the same
 * bits as the job in a mixed launch.  Needs no GPU when the configuration
 * comes from the tune cache or the static resource table.
 */
int ppx_mixed_tile_config(const ppx_job *job, ppx_config *cfg);

/* Most jobs of one family that a launch passes in kernel arguments. */
#define PPX_MIXED_ARG_JOBS 32
/*
 * ppx_mixed_argument_launch -- 1 if launch_mixed would pass these jobs'
 * records in the kernel arguments (no tiled job, or at most
 * PPX_MIXED_ARG_JOBS per family), 0 if it would use the device tables and
 * persistent kernels, or a negative PPX_E* code for jobs it would refuse.
 * Planning only (needs no GPU where ppx_mixed_tile_config needs none).
 */
int ppx_mixed_argument_launch(const ppx_job *jobs, int njobs);

/* ---------------------------------------------------------------------- */
/* Helpers                                                                 */
/* ---------------------------------------------------------------------- */

/* Thread-local message describing the last error ("" if none). */
const char *ppx_last_error(void);

/*
 * ppx_config_valid -- the validity predicate of the search space (Sec. V:
 * the constraints on S, P, L, r and shuffle, restated for gfx950).
 * Returns PPX_OK if cfg describes a launch the library can run for
 * (op, dtype, n), PPX_ECONFIG otherwise (reason in ppx_last_error()).
 * Static check: needs no GPU.
 */
int ppx_config_valid(int op, int dtype, int64_t n, const ppx_config *cfg);

/*
 * ppx_default_config -- the plain per-problem configuration used as the
 * "default" in tuned-vs-default comparisons: one problem per workgroup,
 * radix 2, L = min(n/2, 1024) (FFT) or the smallest L giving P <= 32.
 */
int ppx_default_config(int op, int dtype, int64_t n, ppx_config *out);

/*
 * ppx_resolve_config -- what a call with cfg == NULL will use for
 * (op, dtype, n): the tuned entry if one is cached, else the analytical
 * choice.  Needs no GPU when the analytical choice comes from the static
 * resource table.
 */
int ppx_resolve_config(int op, int dtype, int64_t n, int64_t batch,
                       ppx_config *out);

/*
 * ppx_enumerate_configs -- writes up to `cap` valid configurations for
 * (op, dtype, n) into out[] and returns how many exist (so a call with
 * cap = 0 sizes the array).  Static; needs no GPU.
 */
int ppx_enumerate_configs(int op, int dtype, int64_t n, ppx_config *out,
                          int cap);

#ifdef __cplusplus
}
#endif

#endif /* PPX_H */
