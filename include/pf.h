/*
 * pf.h - C-ABI of libpf_mi355x.so: the fully parallel particle-filter /
 * particle-learning cycle of McAlinn & Nakatsuma, "Parallel Resampling for
 * Fully Parallelized Particle Filters" (arXiv:1212.1639), on one AMD MI355X
 * (gfx950).
 *
 * The problem statement the calls follow is the paper's (Section 2): a state
 * space model y_t ~ p(y_t | x_t, theta), x_t ~ p(x_t | x_{t-1}, theta)
 * (equation (ssm)), a prior for the initial particles, N particles, and
 * observations that arrive one at a time; the outputs are the filtered
 * approximation of the state, posterior statistics of theta (Section 2,
 * after Algorithm "Particle Learning") and the log-likelihood implied by the
 * weight normaliser (equation (pf.resampling)).  As the paper requires
 * (end of Section 3.2), every particle stays in device memory between steps:
 * data cross to the host only when the caller asks for the log-likelihood
 * or the moments.
 *
 * Conventions for every call:
 *   - Return value 0 (PF_OK) or a negative PF_E* code; the text of the last
 *     error of the calling thread is available from pf_last_error().  No C++
 *     exception crosses this interface.
 *   - Pointers named *_dev are device pointers (hipMalloc'd or a torch CUDA
 *     tensor's data_ptr); everything else is host memory.
 *   - A handle is bound to one HIP stream and is not thread-safe; calls on
 *     one handle must not overlap.  pf_step never synchronises the stream.
 *   - Particle and ancestor indices are 0-based.
 */
#ifndef PF_MI355X_H
#define PF_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define PF_OK 0
#define PF_EINVAL (-1)      /* bad argument (message says which)              */
#define PF_ENOMEM (-2)      /* workspace too small or device allocation failed */
#define PF_EDEVICE (-3)     /* a HIP runtime call failed                       */
#define PF_EDEGENERATE (-4) /* every weight of some step was zero or not finite:
                               the normaliser of equation (pf.resampling) is
                               undefined.  Sticky: reported by pf_loglik and
                               pf_moments from then on                         */

/* ---------------------------------------------------------------- models */
/* Local-level ("stochastic trend with noise") model of Section 4, equation
 * (trend+noise): y_t = x_t + v_t, v_t ~ N(0, sigma_v2); x_t = x_{t-1} + w_t,
 * w_t ~ N(0, sigma_w2); x_0 ~ N(x0_mean, x0_var).
 *   PF_LL_PF: known variances, bootstrap filter (Section 2, Algorithm
 *             "Particle Filtering").
 *   PF_LL_PL: unknown variances with priors sigma_v2 ~ IG(a_v, b_v),
 *             sigma_w2 ~ IG(a_w, b_w) (shape, scale), particle learning
 *             (Section 2, Algorithm "Particle Learning", the experiment of
 *             Section 4).
 * Stochastic volatility (not in the paper): x_t = mu + phi (x_{t-1} - mu) +
 * sigma eta_t, y_t ~ N(0, exp(x_t)); x_0 ~ N(x0_mean, x0_var).
 *   PF_SV_PF: known (mu, phi, sigma2), bootstrap filter.
 *   PF_SV_PL: unknown (alpha, beta, sigma^2) = (mu (1 - phi), phi, sigma^2)
 *             with the conjugate prior (alpha, beta) | sigma^2 ~
 *             N(prior_mean, sigma^2 Lambda0^{-1}), sigma^2 ~ IG(a_s, d_s),
 *             learned in the propagate-weight-resample order. */
enum pf_model { PF_LL_PF = 0, PF_LL_PL = 1, PF_SV_PF = 2, PF_SV_PL = 3 };

/* Resampling uniforms (Section 3.1): multinomial i.i.d.; stratified, one per
 * stratum [j/N, (j+1)/N]; systematic, one offset shared by all strata;
 * sorted multinomial, the multinomial scheme with its uniforms formed as
 * order statistics (u_j = P_j / P_N, P_j the sum of the exponential spacings
 * -log U_0 .. -log U_j, U_i from slot i's multinomial word, i = 0..N), so
 * that slots receive ancestors in increasing order and the search merges
 * like the stratified scheme; the offspring counts are multinomial exactly.
 * Sorted multinomial needs the tile scan and is not batched; in PF_FP32 it
 * runs at 1, 2 or 8 items per thread (library choice 2; 4 is refused with
 * PF_EINVAL). */
enum pf_scheme {
    PF_MULTINOMIAL = 0,
    PF_STRATIFIED = 1,
    PF_SYSTEMATIC = 2,
    PF_SORTED_MULTINOMIAL = 3
};

/* Arithmetic of states and weights.  The CDF tile sums, normaliser and
 * log-likelihood are always accumulated in double precision. */
enum pf_precision { PF_FP32 = 0, PF_FP64 = 1 };

/* How the inverse CDF a_j = min{k : q(k) >= u_j} is found (Section 3.2).
 * Every strategy returns the same ancestors for the same CDF and uniforms.
 *   PF_SEARCH_AUTO:     library choice (merge for sorted uniforms; for
 *                       multinomial uniforms the cut-point method, except
 *                       that a CDF of 2049 to 512 x items_per_thread
 *                       entries, which fits one LDS window but not the LDS
 *                       cut-point table, merges).
 *   PF_SEARCH_BINARY:   bisection per uniform.
 *   PF_SEARCH_CUTPOINT: the paper's parallel cut-point method: table
 *                       I_k = min{i : q(i) > (k-1)/N} built by the
 *                       parallelized cut-point search, then a climb from
 *                       I_{ceil(N u)}; the climb is bounded, falling back
 *                       to bisection above the start point.  Up to
 *                       min(2048, 512 x items_per_thread) particles the
 *                       table is built in each work-group's LDS; above, it
 *                       lives in the workspace (4 bytes per particle) and
 *                       is built by a launch of its own after each
 *                       weighting, from an upper envelope of ceil(N q(i))
 *                       that keeps every start at or below the answer
 *                       (needs the default tile scan, not
 *                       PF_FLAG_LOOKBACK_SCAN).
 *   PF_SEARCH_MERGE:    work-group cooperative merge of sorted uniforms
 *                       against the CDF staged in LDS. */
enum pf_strategy {
    PF_SEARCH_AUTO = 0,
    PF_SEARCH_BINARY = 1,
    PF_SEARCH_CUTPOINT = 2,
    PF_SEARCH_MERGE = 3
};

/* PF_FLAG_KEEP_ANCESTORS: also store each step's ancestor indices (4 bytes
 * per particle per step) so pf_debug_particles can return them; off by
 * default because the cycle itself never reads them back. */
#define PF_FLAG_KEEP_ANCESTORS 1
/* PF_FLAG_LOOKBACK_SCAN: form the CDF's tile prefixes in the cycle kernel
 * itself by a decoupled look-back over the tiles' (max, sum) aggregates,
 * instead of the default: tiles store their (max, sum) and one extra
 * work-group scans them in a fixed order.  Both give the same CDF up to
 * rounding; the default is deterministic and faster on MI355X. */
#define PF_FLAG_LOOKBACK_SCAN 2
/* PF_FLAG_TEST_SCAN_STALL: a test aid for the bounded waits of the tile
 * scans run inside the cycle kernel (the look-back, and the scan of filters
 * of at most 16 tiles in the kernel's last work-group): every such wait
 * looks for words no tile writes and gives up after 64 polls, as it would
 * if a tile never published its sums.  The launches end normally; the next
 * pf_loglik or pf_moments reports PF_EDEVICE.  The filter's results are
 * meaningless.  (Without it a wait gives up after 2^22 polls.) */
#define PF_FLAG_TEST_SCAN_STALL 4

typedef struct pf_config {
    int32_t model;            /* enum pf_model                                 */
    int32_t scheme;           /* enum pf_scheme                                */
    int32_t precision;        /* enum pf_precision                             */
    int32_t strategy;         /* enum pf_strategy                              */
    int64_t n_particles;      /* N >= 1 and N <= 2^31 - 1                       */
    uint64_t seed;            /* key of the counter-based generator             */
    int32_t items_per_thread; /* 0 = library choice, else one of 1, 2, 4, 8
                                 (4 is refused, PF_EINVAL, for PF_SV_PL in
                                 PF_FP64: switched off, its kernel gave wrong
                                 weights; the library choice there is 1; and
                                 for PF_SORTED_MULTINOMIAL in PF_FP32, whose
                                 library choice is 2)                         */
    int32_t flags;            /* bitwise OR of PF_FLAG_*; other bits must be 0  */
    double x0_mean, x0_var;   /* prior of x_0                                  */
    double sigma_v2, sigma_w2;/* PF_LL_PF: known variances                     */
    double a_v, b_v, a_w, b_w;/* PF_LL_PL: inverse-gamma priors                */
    double mu, phi, sigma2;   /* PF_SV_PF: known parameters                    */
    double prior_mean[2];     /* PF_SV_PL: mean of (alpha, beta) given sigma^2  */
    double prior_prec[3];     /* PF_SV_PL: Lambda0 = [[p0, p1], [p1, p2]], SPD  */
    double a_s, d_s;          /* PF_SV_PL: inverse-gamma prior of sigma^2       */
} pf_config;

typedef struct pf_filter pf_filter;

/* Number of values each particle keeps in device memory for `model`
 * (the record layout of pf_debug_particles); 0 for an unknown model. */
int pf_fields(int32_t model);

/* Device bytes a filter with this configuration needs: particle records
 * (double-buffered, structure of arrays), the CDF, per-tile scan state and
 * a few scalars.  0 if the configuration is invalid (see pf_last_error). */
size_t pf_workspace_bytes(const pf_config* cfg);

/* Create a filter and sample its initial particles (Step 0 of both
 * algorithms of Section 2) on `hip_stream` (NULL = the null stream).
 *   workspace_dev: caller-owned device memory of at least
 *       pf_workspace_bytes(cfg) bytes, 256-byte aligned, that outlives the
 *       handle; NULL makes the library allocate (and later free) it.
 *   out: receives the handle.
 * Errors: PF_EINVAL (bad configuration, misaligned workspace), PF_ENOMEM
 * (ws_bytes too small, allocation failed), PF_EDEVICE. */
int pf_create(const pf_config* cfg, void* workspace_dev, size_t ws_bytes, void* hip_stream,
              pf_filter** out);

/* Assimilate n_obs >= 1 observations y[0..n_obs-1] (host memory, read
 * before the call returns) in order: for each one, a full cycle of weights,
 * CDF, resampling and propagation runs on the device (Section 3.2: the whole
 * cycle is parallel).  Asynchronous with respect to the host.  Errors:
 * PF_EINVAL (n_obs < 1, a non-finite observation: nothing is launched),
 * PF_EDEVICE. */
int pf_step(pf_filter* f, const double* y, int64_t n_obs);

/* Synchronise the filter's stream and return in *out the log-likelihood
 * estimate sum_t log( (1/N) sum_i p(y_t | particle i) ) over the
 * observations assimilated so far (0 before any).  Errors: PF_EDEGENERATE,
 * PF_EDEVICE (also when a filter of at most 16 tiles, whose tile scan runs
 * in the cycle kernel's last work-group, found a tile's sums missing after
 * its bounded wait; sticky like PF_EDEGENERATE). */
int pf_loglik(const pf_filter* f, double* out);

/* Synchronise and return posterior statistics of the latest time step in
 * out[0..n-1], n = the model's count (PF_LL_PF, PF_SV_PF: 3; PF_LL_PL: 6;
 * PF_SV_PL: 7); n_out must be >= n, extra entries are set to 0.
 *   PF_LL_PF, PF_SV_PF (weights of the latest step, before resampling):
 *     [E x_t, Var x_t, effective sample size].
 *   PF_LL_PL (equal weights, after propagation):
 *     [E x_t, Var x_t, mean of drawn sigma_v2, mean of drawn sigma_w2,
 *      Rao-Blackwell mean b_v/(a_v - 1), Rao-Blackwell mean b_w/(a_w - 1)]
 *     (no effective sample size: with equal weights it is N).
 *   PF_SV_PL (weights of the latest step):
 *     [E x_t, Var x_t, E alpha, E beta, E sigma^2 of the draws,
 *      effective sample size, Rao-Blackwell mean of sigma^2].
 * For PF_LL_PL this may launch the propagation of the latest observation
 * (the cycle weights y_{t+1} before it propagates with y_t).  Errors:
 * PF_EINVAL, PF_EDEGENERATE, PF_EDEVICE (as pf_loglik). */
int pf_moments(pf_filter* f, double* out, int32_t n_out);

/* Release a handle and, if the library allocated it, its workspace.
 * NULL is accepted.  Synchronises the stream first. */
int pf_destroy(pf_filter* f);

/* Text of the calling thread's last error ("" if none). */
const char* pf_last_error(void);

/* ---------------------------------------------------------- batches  */
/* Many independent filters stepped together (the cycle of Section 3.2 run
 * for all of them at once): per observation, one launch works
 * through the tiles of every filter in the batch and one launch scans each
 * filter's tiles; the pair is captured once in a HIP graph and replayed per
 * step, its arguments read from a device ring filled ahead of time.  A
 * filter's results are the same as when it is stepped alone, bit for bit. */
typedef struct pf_batch pf_batch;

/* Group n >= 1 distinct filters of one model, precision and
 * items_per_thread, all using the default tile scan.  capacity (>= n; less
 * means n) bounds the membership pf_batch_update may set later.  The batch
 * launches on the first filter's stream; the filters keep their own
 * workspaces and must not be stepped on their own while they are members
 * (pf_loglik, pf_moments and pf_debug_particles on them remain valid).  ring
 * (0 = 64) is how many steps' arguments one pf_batch_step call can queue at
 * once.  Errors: PF_EINVAL, PF_ENOMEM, PF_EDEVICE. */
int pf_batch_create(pf_filter* const* filters, int32_t n, int32_t capacity, int32_t ring,
                    pf_batch** out);

/* Replace the members (0 <= n <= capacity; same model, precision and
 * items_per_thread as at creation).  Filters may join at any stage and leave
 * at any time; the batch's captured graph stays valid.  Ordered on the
 * batch's stream.  Errors: PF_EINVAL, PF_EDEVICE. */
int pf_batch_update(pf_batch* b, pf_filter* const* filters, int32_t n);

/* Advance every member by n_steps observations: y[s * n + f] (host memory,
 * read before return) is member f's observation at step s (n = current
 * members; nothing happens when there are none).  Asynchronous.
 * Errors: PF_EINVAL (n_steps < 1, a non-finite observation: nothing is
 * launched), PF_EDEVICE. */
int pf_batch_step(pf_batch* b, const double* y, int64_t n_steps);

/* Device bytes a batch allocates for itself (beyond its members'
 * workspaces) with this capacity and ring (ring < 1 means 64) when its
 * members hold `tiles` tiles in all: the ring of per-step member arguments,
 * the member table, the global tile map and the batch's progress counters.
 * A memory budget that admits filters by pf_workspace_bytes charges this
 * too.  0 for capacity < 1 or tiles < 0.  Host-only (no device call). */
size_t pf_batch_bytes(int32_t capacity, int32_t ring, int64_t tiles);

/* Release a batch (not its filters).  NULL is accepted. */
int pf_batch_destroy(pf_batch* b);

/* One step of n filters as a batch: the same as pf_batch_create (capacity
 * n, ring 1), pf_batch_step(.., y_each, 1) and pf_batch_destroy. */
int pf_step_batch(pf_filter* const* filters, int32_t n, const double* y_each);

/* ------------------------------------------------------- test surfaces  */
/* Inverse-CDF search alone (Section 3.2), the exact-parity surface of the
 * resampling step: anc_dev[j] = min{k : cdf_dev[k] >= u_dev[j]}, or n-1 when
 * no entry reaches u_dev[j].
 *   cdf_dev: n >= 1 non-decreasing doubles (checked on the device:
 *            PF_EINVAL if decreasing anywhere or not finite);
 *   u_dev:   m >= 0 doubles in (0, 1];  anc_dev: m int32 outputs;
 *   strategy: PF_SEARCH_BINARY, PF_SEARCH_CUTPOINT or PF_SEARCH_MERGE
 *            (AUTO = MERGE).  Synchronises the stream before returning.
 * n must be <= 2^31 - 1.  Errors: PF_EINVAL, PF_ENOMEM, PF_EDEVICE. */
int pf_debug_search(const double* cdf_dev, const double* u_dev, int64_t n, int64_t m,
                    int32_t strategy, int32_t* anc_dev, void* hip_stream);

/* pf_debug_search for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and results, but the check flag and the
 * cut-point table live in a static device array that each GPU holds for
 * the life of the process (4 MiB + 256 B), so no call allocates or frees.
 * The table holds at most 2^20 entries: PF_SEARCH_CUTPOINT with
 * n > 2^20 is PF_EINVAL (the other strategies take any n < 2^31).  The
 * array of the current device is used (hip_stream must belong to it) and
 * every call on that device shares it: calls that overlap on one GPU, from
 * several threads or streams, race.  Synchronises the stream.  Errors as
 * pf_debug_search, without PF_ENOMEM. */
int pf_debug_search_noalloc(const double* cdf_dev, const double* u_dev, int64_t n, int64_t m,
                            int32_t strategy, int32_t* anc_dev, void* hip_stream);

/* Copy the current particles to host memory for small-N tests: the record
 * as pf_fields(model) arrays of N values (float for PF_FP32, double for
 * PF_FP64), followed by N int32 ancestors that produced them (identity when
 * no resampling happened; all -1 unless the filter was created with
 * PF_FLAG_KEEP_ANCESTORS).  bytes must be >= that size.  *t_out (if not
 * NULL) receives the number of propagations done so far.  Synchronises.
 * Record fields: PF_LL_PF, PF_SV_PF: x.  PF_LL_PL: x, b_v, b_w, sigma_v2,
 * sigma_w2.  PF_SV_PL: x, L01, L11, eta0, eta1, d, where Lambda = [[L00,
 * L01], [L01, L11]] and eta are the precision and the precision-weighted
 * mean of the (alpha, beta) posterior and d its inverse-gamma scale
 * (L00 = p0 + t and the shape a_s + t/2 are the same for every particle). */
int pf_debug_particles(pf_filter* f, void* host_out, size_t bytes, int64_t* t_out);

/* Copy the current particles' record (pf_fields(model) arrays of N
 * values, float for PF_FP32 and double for PF_FP64, as pf_debug_particles
 * lays them out, without the ancestors) to host memory asynchronously: the
 * copy is queued on copy_stream (a hipStream_t; NULL = the null stream)
 * after f's latest launch, and f's next launch that would overwrite those
 * particles (two propagations later: the record is double-buffered) first
 * waits for the copy, so stepping continues while the copy runs.  host_dst
 * (caller-owned, at least bytes >= fields * N * element size) should be
 * pinned (hipHostMalloc) for the copy to be asynchronous; its contents are
 * valid once copy_stream has passed the copy.  This is the "store the
 * particles in host memory" phase of the paper's experiment (Section 4),
 * overlapped with the next step.  Errors: PF_EINVAL, PF_EDEVICE.
 * CURRENTLY SWITCHED OFF: the call returns PF_EDEVICE without doing anything
 * (its first GPU run faulted; the cause is not yet found).  Use
 * pf_debug_particles for a synchronous copy. */
int pf_copy_particles_async(pf_filter* f, void* host_dst, size_t bytes, void* copy_stream);

/* ------------------------------------------------------ checkpoints  */
/* Snapshot and resume of a filter's state, so that a server can pre-empt a
 * filter (free its device memory) and later continue it.  Everything the
 * next cycle reads is kept: the current particle record, the latest CDF
 * (in-tile prefixes, tile tables, totals, cut-point table), the running
 * log-likelihood, moment partials and error flags, and the host-side step
 * state (time index, buffer parity, a particle-learning filter's pending
 * observation).  The random draws are counter-based on (seed, slot, time),
 * so a restored filter continues exactly as the uninterrupted one would,
 * bit for bit with the default tile scan (Section 3.2's cycle is a function
 * of the particles, the CDF and the step's draws).
 *
 * pf_checkpoint_bytes: host bytes a snapshot of f takes (0 for NULL); it
 *   does not change while the filter steps.
 * pf_checkpoint_save: synchronise f's stream and write the snapshot into
 *   host_out (caller-owned, bytes >= pf_checkpoint_bytes(f)).  Layout: a
 *   fixed header (format tag, the configuration, the host-side state)
 *   followed by the workspace minus the two buffers the next cycle
 *   overwrites without reading.  Errors: PF_EINVAL, PF_EDEVICE.
 * pf_checkpoint_restore: load a snapshot into f, which must have been
 *   created with the same configuration (model, scheme, precision, N, seed,
 *   flags, parameters, and the same resolved tile size and strategy);
 *   f's own state is replaced.  f must not be a member of a batch with
 *   steps queued.  Synchronises f's stream.  Errors: PF_EINVAL (not a
 *   snapshot, another configuration, truncated), PF_EDEVICE. */
size_t pf_checkpoint_bytes(const pf_filter* f);
int pf_checkpoint_save(pf_filter* f, void* host_out, size_t bytes);
int pf_checkpoint_restore(pf_filter* f, const void* host_in, size_t bytes);

/* Autotuner (a runtime aid, not part of the method): picks the tile size
 * (cfg->items_per_thread), the search strategy (cfg->strategy) and the CDF
 * scan (the PF_FLAG_LOOKBACK_SCAN bit of cfg->flags) for cfg by timing
 * candidates on hip_stream: first items_per_thread in {1, 2, 4, 8} with the
 * library's default strategy and the tile scan, then every strategy valid at
 * the best tile size, then the look-back scan.  Each candidate is a
 * temporary filter (library-allocated workspace) stepped over y[0..n_obs)
 * (host array, n_obs >= 3; the first two steps are warm-up).  Other fields
 * of *cfg are kept; the choice is written back into *cfg and cached per
 * (device, model, precision, scheme, ancestor flag, ceil(log2 N)), so a later
 * call for a similar configuration returns at once.  *ms_per_step (if not
 * NULL) receives the winner's time per step.  Synchronises hip_stream.
 * The random draws do not depend on the choice; the CDF's summation order
 * (tile boundaries) does, so results agree to rounding.  Errors: PF_EINVAL
 * (invalid cfg, n_obs < 3, non-finite y), PF_ENOMEM (no candidate fits),
 * PF_EDEVICE. */
int pf_autotune(pf_config* cfg, const double* y, int64_t n_obs, void* hip_stream,
                double* ms_per_step);

/* Autotuner of a batch: the common items_per_thread in {1, 2, 4, 8} (with
 * the default strategy), then bisection instead of the default search at
 * that size, timed by stepping temporary copies of the n filters cfgs[0..n)
 * as one batch (pf_batch_step) over y[s * n + f], s < n_obs (n_obs >= 3).
 * Writes items_per_thread and strategy into every cfgs[k]; batched filters
 * use the tile scan (PF_FLAG_LOOKBACK_SCAN set is PF_EINVAL).  Not cached.
 * Synchronises hip_stream.  Errors as pf_autotune. */
int pf_autotune_batch(pf_config* cfgs, int32_t n, const double* y, int64_t n_obs,
                      void* hip_stream, double* ms_per_step);

/* Kernel timing, a measurement aid (not part of the method).
 * pf_timing_start synchronises f's stream and arms max_launches
 * (1 <= max_launches <= 2^20) pairs of HIP events: of f's next cycle-kernel
 * launches, the 1st, (every+1)-th, (2 every+1)-th, ... (every >= 1), up to
 * max_launches of them, are each bracketed by one pair on f's stream (the
 * CDF tile scan that follows a weighting launch is outside the bracket);
 * bracketing one launch in `every` keeps the events' own cost out of the
 * other launches.  pf_timing_read synchronises, returns in *total_ms the
 * summed event-to-event time of the bracketed launches and in *launches
 * their count, and disarms.  Arming again discards earlier pairs.  The
 * events are owned by the handle and released by pf_timing_read or
 * pf_destroy.  Errors: PF_EINVAL (null argument, bad count), PF_EDEVICE. */
int pf_timing_start(pf_filter* f, int64_t max_launches, int64_t every);
int pf_timing_read(pf_filter* f, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* PF_MI355X_H */
