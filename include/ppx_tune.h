/*
 * ppx_tune.h -- the tuning engine behind tune() (include/ppx.h), exposed so
 * that each part can be driven with a caller-supplied evaluator or device
 * model (no GPU needed for anything here except ppx_tune_ex and
 * ppx_kernel_resources).
 *
 * Source: arXiv:2310.16214, Sec. IV-A (premises of the analytical model:
 * warp occupancy W_SM against W^max and active blocks B_a against B^max;
 * the four-step guideline), Fig. "analytical-tuning"(a) (the GM20B
 * occupancy table the model must reproduce), Sec. IV-B (Bayesian
 * optimisation: random initial samples, surrogate, Expected Improvement,
 * stop after no progress in the last 5 evaluations, invalid or overlong runs
 * get a high time), Sec. VI (exhaustive search as the reference; the
 * harmonic-mean Phi metric).
 *
 * All functions return PPX_OK or a negative PPX_E* code (ppx_last_error()).
 */
#ifndef PPX_TUNE_H
#define PPX_TUNE_H

#include <stdint.h>

#include "ppx.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Occupancy model of one compute unit (CU / SM).  Registers are counted as
 * 32-bit lane slots: a wave of `wave_size` lanes using R registers per lane
 * occupies roundup(R * wave_size, reg_granule) slots of one partition.
 *   gfx950:  wave 64, 4 SIMD partitions of 512 VGPRs x 64 lanes = 32768
 *            slots, granule 8 VGPRs x 64 = 512, 32 waves / CU, 32 blocks /
 *            CU, 160 KiB LDS per CU and per block.
 *   GM20B:   warp 32, 4 partitions of 16384 registers, granule 256, 64
 *            warps / SM, 32 blocks / SM, 64 KiB shared per SM, 48 KiB per
 *            block (Sec. II).
 */
typedef struct ppx_device_model {
    int32_t wave_size;
    int32_t partitions;
    int32_t regs_per_partition;
    int32_t reg_granule;
    int32_t max_waves_per_cu;   /* W^max */
    int32_t max_blocks_per_cu;  /* B^max */
    int32_t lds_per_cu;
    int32_t lds_per_block;
    int32_t lds_granule;
    int32_t num_cus;
} ppx_device_model;

/* Resources of one candidate launch. */
typedef struct ppx_resource {
    int32_t threads;          /* L */
    int32_t regs_per_thread;  /* VGPRs (gfx950) or registers (GM20B) */
    int32_t lds_bytes;        /* per block, static + dynamic */
} ppx_resource;

/* Occupancy of a candidate: blocks = B_a, waves = W_SM = B_a * waves/block.
 * Returns PPX_ECONFIG (blocks = waves = 0) if the block cannot run at all. */
int ppx_occupancy(const ppx_device_model *m, const ppx_resource *r, int32_t *blocks,
                  int32_t *waves);

/* The gfx950 model: the current device's limits if a device has been
 * initialised in this process, else the published MI355X figures. */
int ppx_device_model_gfx950(ppx_device_model *out);

/*
 * Analytical guideline (Sec. IV-A) over `ncands` candidates with their
 * resources.  Steps: (1) candidates reaching W_SM = W^max and B_a = B^max;
 * else (2) the largest B_a with W_SM / W^max in [60%, 100%]; else (3) the
 * largest warp occupancy, ties to the larger P; and (4) within steps 1-2 a
 * larger radix wins even at a lower B_a.  `flags`:
 *   PPX_ANALYTICAL_GRID_FILL  (gfx950 term, ours) first keep only the
 *       candidates whose grid ceil(batch / G_b) fills every CU with B_a
 *       blocks, when any does;
 *   PPX_ANALYTICAL_WINDOW_50 (gfx950 term, ours) lower the occupancy window
 *       of steps 1-2 from 60% to 50% of W^max (four waves per SIMD).
 * Writes the chosen index to *chosen.  The library's own analytical choice
 * (tune() with PPX_TUNE_ANALYTICAL, and a NULL config with nothing tuned)
 * uses GRID_FILL | WINDOW_50 over the candidates whose global accesses are
 * coalesced per instruction (for the scan: P <= 4, one 16-byte vector per
 * lane).
 */
#define PPX_ANALYTICAL_GRID_FILL 1
#define PPX_ANALYTICAL_WINDOW_50 4
int ppx_analytical_pick(const ppx_device_model *m, const ppx_config *cands,
                        const ppx_resource *res, int ncands, int64_t batch, int flags,
                        int *chosen);

/*
 * The library's analytical choice (what tune() with PPX_TUNE_ANALYTICAL
 * picks: the gfx950 candidate rules, the occupancy guideline with grid fill
 * and the 50% window, and the persistent twin of a choice that keeps at most
 * two workgroups resident) restricted to a caller's candidate list, e.g. a
 * smaller search space.  Each candidate must be valid for (op, dtype, n);
 * *chosen receives the index of the choice.  Resources come from the device
 * when one is initialised, else from the static table.
 */
int ppx_analytical_select(int op, int dtype, int64_t n, int64_t batch, const ppx_config *cands,
                          int ncands, int *chosen);

/*
 * Consistency check of the mixed launch (launch_mixed): PPX_OK if every
 * family of tile shapes has its persistent kernel in the library, else
 * PPX_EINVAL naming the first family without one.  Needs no GPU.
 */
int ppx_mixed_families_complete(void);

/* Evaluator: the cost (e.g. median microseconds) of a candidate; a negative
 * value marks a failed or timed-out run. */
typedef double (*ppx_eval_fn)(const ppx_config *cfg, void *user);

/*
 * Bayesian-optimisation search (Sec. IV-B) over a finite candidate list.
 * Surrogate: Gaussian process on log-cost with a Matern-5/2 ARD kernel over
 * the features (log2 r, log2 L, log2 G_b, algo) scaled to [0, 1], signal and
 * noise variances and length scales fitted by maximum marginal likelihood
 * (multi-start Nelder-Mead in log space).  Acquisition: Expected Improvement,
 * maximised by enumeration over the unevaluated candidates.  n_init seeded
 * random candidates first (n_init <= 0: max(3, ceil(5% of ncands))).  Stops
 * when the last `patience` evaluations (<= 0: 5) brought no improvement
 * larger than `min_rel_improvement` (relative, on cost), when every candidate
 * is evaluated, or after max_evals (<= 0: no cap).  A failed evaluation is
 * recorded at 10x the worst cost observed so far.
 *   order_out[i]  index of the i-th evaluated candidate (capacity ncands)
 *   values_out[i] its cost as recorded (capacity ncands)
 */
int ppx_bo_search(const ppx_config *cands, int ncands, ppx_eval_fn fn, void *user,
                  int max_evals, int n_init, int patience, double min_rel_improvement,
                  uint64_t seed, int *order_out, double *values_out, int *evals_used,
                  int *best_index);

/* GP posterior mean and variance of the latent function at m query points,
 * for a Matern-5/2 ARD kernel k = sigma_f2 * (1 + s + s^2/3) exp(-s),
 * s = sqrt(5) * ||(x - x') / lengthscales||, observation noise noise2.
 * X: n x d, Xq: m x d, row-major. */
int ppx_gp_posterior(const double *X, const double *y, int n, int d,
                     const double *lengthscales, double sigma_f2, double noise2,
                     const double *Xq, int m, double *mean, double *var);

/* Expected improvement of a minimisation at a point with posterior mean mu and
 * standard deviation sigma, given the best value so far. */
double ppx_expected_improvement(double mu, double sigma, double best);

/* Per-candidate report of a GPU tuning run. */
typedef struct ppx_tune_report {
    ppx_config best;
    double best_us;
    int32_t evals_used;
    int32_t ncands;          /* size of the valid space */
    ppx_config *trace_cfg;   /* optional (capacity trace_cap): evaluated configs */
    double *trace_us;        /* their median microseconds (<0: failed) */
    int32_t trace_cap;
} ppx_tune_report;

/*
 * ppx_tune_ex -- tune() with an algorithm filter and a full report.  algo =
 * -1 searches every algorithm of the op; otherwise only that one (the cache
 * entry is then keyed by it); for the tridiagonal solvers the filter selects
 * a family: PPX_TRI_CR (CR through LDS or shuffles), PPX_TRI_PCR (the PCR
 * variants), PPX_TRI_CR_PCR (the hybrid), PPX_TRI_WM or PPX_TRI_LF.  reps = timed launches per candidate (<= 0:
 * 100, the paper's count), each on a different buffer set so that no rep
 * reads data a previous rep left in the 256 MB Infinity Cache.  Synchronous;
 * needs a GPU.  Records the winner in the tune cache.
 */
int ppx_tune_ex(int op, int dtype, int64_t n, int64_t batch, int method, int max_evals,
                int algo, int reps, ppx_tune_report *report);

/*
 * ppx_tune_large_trace -- tune_fft_large with `reps` timed launches per plan
 * (<= 0: 100) and the timed plans in evaluation order: up to trace_cap
 * entries of trace_plan / trace_us (either may be NULL).  Returns the number
 * of timed plans (>= 0) or a negative PPX_E* code.  Needs a GPU.
 */
int ppx_tune_large_trace(int64_t n, int64_t batch, int method, int max_evals, int reps, ppx_fft_plan *best,
                         double *best_us, int *evals_used, ppx_fft_plan *trace_plan, double *trace_us,
                         int trace_cap);

/*
 * Online tuning session -- the learned search of Sec. IV-B run one
 * evaluation at a time, for callers (a request loop) that time candidates on
 * their own launches and amortise the evaluations over repeated requests of
 * one (op, dtype, n): the online use the paper's conclusion recommends the
 * learned tuner for.  Candidates: as ppx_tune_ex (algo = -1: all, else one
 * algorithm or tridiagonal family); the same BO state, seed and stopping rule
 * as ppx_tune_ex's learned method, with max_evals (<= 0: no cap).  Costs are
 * in any unit where lower is better.  Host-only bookkeeping: no GPU work.
 * A session is not thread-safe.
 *
 * ppx_online_create   batch: a typical batch, for the analytical
 *                     configuration used before any evaluation.
 * ppx_online_next     *cfg receives the configuration for the next launch.
 *                     Returns 1 when it is a candidate whose cost must be
 *                     reported (ppx_online_report) before another is
 *                     proposed; 0 when it is the session's current choice
 *                     (best evaluated so far, else the analytical one):
 *                     with explore == 0, while a cost is awaited, or once
 *                     the search has stopped.  Negative on error.
 * ppx_online_report   the pending candidate's cost (negative: it failed).
 * ppx_online_status   evaluations so far, whether the search has stopped,
 *                     the current choice and its cost (-1 before any).
 */
typedef struct ppx_online ppx_online;
int ppx_online_create(int op, int dtype, int64_t n, int64_t batch, int algo, int max_evals,
                      ppx_online **out);
int ppx_online_next(ppx_online *o, int explore, ppx_config *cfg);
int ppx_online_report(ppx_online *o, double cost);
int ppx_online_status(const ppx_online *o, int *evals, int *converged, ppx_config *best,
                      double *best_cost);
int ppx_online_destroy(ppx_online *o);

/* Median microseconds of `reps` launches of one explicit configuration, timed
 * like a tuning candidate (the default-vs-tuned baseline uses this). */
int ppx_time_config(int op, int dtype, int64_t n, int64_t batch, const ppx_config *cfg,
                    int reps, double *median_us);

/* Resources of the kernel behind a configuration on the current device
 * (hipFuncGetAttributes). */
int ppx_kernel_resources(int op, int dtype, int64_t n, const ppx_config *cfg,
                         ppx_resource *out);

/*
 * ppx_stream_reference -- measurement reference, not part of the method: a
 * plain streaming kernel that reads k in [1, 4] input arrays of `bytes` bytes
 * each and writes their element-wise float sum (16-byte accesses, one per
 * thread) to `out`.  It moves exactly the HBM bytes of a batched call with k
 * input streams and one output stream, so its rate is the practical ceiling
 * that a call of that size and pattern can reach.  in[0..k-1], out: device
 * pointers, 16-byte aligned; bytes > 0, a multiple of 16, at most 2^36.
 * Asynchronous on `stream`; PPX_EINVAL on bad arguments.
 */
int ppx_stream_reference(const void *const *in, int k, void *out, int64_t bytes, void *stream);

/*
 * Tune cache: tuned configurations keyed by (op, dtype, n, algo filter) for
 * the running device architecture, and tuned large-FFT plans keyed by n.
 * Text file, one entry per line:
 *   arch op dtype n algo radix P L G_b S algo_cfg us method
 *   arch plan n log2_n1 radix_a radix_b tile_a tile_b us method
 * load merges the file into memory (returns the number of entries taken;
 * entries no longer valid are skipped); save writes every entry; clear
 * empties both kinds.
 */
int ppx_tune_cache_load(const char *path);
int ppx_tune_cache_save(const char *path);
int ppx_tune_cache_clear(void);
/* Cached entry for (op, dtype, n, algo filter); PPX_EINVAL if none. */
int ppx_tuned_config(int op, int dtype, int64_t n, int algo, ppx_config *out);
/* Tuned large-FFT plan for n (fft_batched_large's plan == NULL uses it);
 * PPX_EINVAL if none. */
int ppx_tuned_fft_plan(int64_t n, ppx_fft_plan *out);

#ifdef __cplusplus
}
#endif

#endif /* PPX_TUNE_H */
