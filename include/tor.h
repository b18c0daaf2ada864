/*
 * tor.h -- C ABI of the MI355X (gfx950) library for exact threshold-detector
 * Gaussian boson sampling probabilities.
 *
 * Method (arXiv:1810.00900, Sec. II "The Algorithm"): the POVM element of a
 * click, I - |0><0|, is a difference of two Gaussian operators, so by
 * linearity the probability of a click pattern is a signed sum, over the
 * subsets Y of the clicked modes C, of Gaussian vacuum probabilities
 *
 *     p(C, N) = sum_{Y subset of C} (-1)^{|Y|} det(sigma_Q[Y u N])^{-1/2}
 *             = P_vac(N) * sum_{Y subset of C} (-1)^{|Y|} det(Sigma_C[Y])^{-1/2},
 *
 * where sigma_Q = sigma + I/2 (hbar = 1), N are the no-click modes, P_vac(N) =
 * det(sigma_Q[N])^{-1/2} is the q_k of Eq. (prob) at zero mean, and Sigma_C is
 * sigma_Q[C] conditioned on vacuum at N (the Schur complement of Eq.
 * MatrixUpdate applied for every mode of N).  Equivalently
 * p = P_vac(N) det(Sigma_C)^{-1/2} Tor(O), O = I - Sigma_C^{-1}, with the
 * Torontonian Tor(O) = sum_{Z subset of C} (-1)^{n-|Z|} det(I - O_Z)^{-1/2}.
 *
 * Conventions shared by every entry point:
 *   cov      host pointer, 2m x 2m, row-major binary64, quadratures interleaved
 *            per mode (x1, p1, x2, p2, ...) as in the paper's quadrature vector
 *            (Sec. II, Eq. 1), hbar = 1 (vacuum = I/2; the paper's hbar = 2
 *            covariance is V = 2 cov), zero mean.  Must be finite and symmetric
 *            to 1e-12 relative; only the lower triangle enters the arithmetic.
 *   pattern  host pointer, int8[m]: 1 = click, 0 = no click, -1 = unobserved
 *            (traced out).  At most TOR_MAX_CLICKS entries may be 1.
 *   sigma_Q  formed as sigma + I/2 exactly (double-double), so the result is
 *            that of the binary64 input matrix.
 *
 * Precision: the 2^n-term alternating sum cancels heavily (the cancellation
 * ratio R = sum|terms| / |sum| reaches 1e10-1e20 at n = 16-28 on 800-mode
 * states), and the paper reports quad precision was needed (Sec. III,
 * "Memory").  The sum is always accumulated in double-double.  The per-subset
 * factorisation runs in binary64 (TOR_PREC_F64) or in double-double
 * (TOR_PREC_DD); TOR_PREC_AUTO runs binary64 first and repeats in
 * double-double when the a-priori bound exceeds tol.  TOR_PREC_QD (opt-in;
 * tor_probability, tor_probability_displaced, tor_subset_sum, tor_batch and
 * tor_batch_displaced (one query at a time) and gbs_chain_fixed) runs the
 * no-click conditioning,
 * the factorisation and the sum in quad-double (about 212 bits): for sums
 * that cancel beyond double-double, e.g. full patterns conditioned on
 * hundreds of no-click modes (R ~ 1e36 at n = 28 on 800 modes).  Its trees
 * use 8-mode wave tasks (7-mode with a mean row) and need about 5.5 GB of
 * device memory at n = 28 (x 2 per further click).  Displaced states take
 * the per-query conditioning route in quad-double (an inverted state's
 * inverse serves binary64 and double-double terms).
 *
 * Status codes: 0 = TOR_OK; TOR_WARN_PRECISION (1): result delivered but its
 * error bound exceeds tol; negative values are errors and leave *out
 * unspecified.  tor_last_error() returns a thread-local message for the last
 * failing call on the calling thread.
 *
 * Ownership: the caller owns every buffer passed in; the library copies
 * inputs before returning.  tor_ctx and tor_state objects are library-owned and
 * freed by their destroy calls; a state must not outlive its context.  A
 * context is not thread-safe: use one per thread or lock externally.
 */
#ifndef TOR_H
#define TOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tor_status;
#define TOR_OK 0
#define TOR_WARN_PRECISION 1
#define TOR_EINVAL (-1)  /* bad argument (null pointer, bad pattern value, not symmetric, NaN) */
#define TOR_ENOTPD (-2)  /* a pivot of sigma_Q was not positive: not a physical covariance */
#define TOR_ETOOBIG (-3) /* more than TOR_MAX_CLICKS clicks, or m too large */
#define TOR_ENOMEM (-4)  /* device or host allocation failed */
#define TOR_EDEVICE (-5) /* HIP runtime error (message in tor_last_error) */
#define TOR_EAGAIN (-6)  /* not ready / not admitted yet */

#define TOR_MAX_CLICKS 32

typedef enum { TOR_PREC_AUTO = 0, TOR_PREC_F64 = 1, TOR_PREC_DD = 2, TOR_PREC_QD = 3 } tor_prec;

typedef struct tor_ctx tor_ctx;
typedef struct tor_state tor_state;

typedef struct {
    double p;             /* click-pattern probability p(C, N) (binary64 rounding of p_hi + p_lo) */
    double p_lo;          /* low word: p + p_lo is the double-double result */
    double log_p;         /* natural log of p (-inf if p <= 0) */
    double tor;           /* Torontonian Tor(I - Sigma_C^-1) = det(Sigma_C)^{1/2} * T */
    double T;             /* subset sum over Sigma_C (= p / P_vac(N)) */
    double T_lo;          /* low word of T */
    double abs_sum;       /* sum of |terms| over Sigma_C */
    double cancel_ratio;  /* abs_sum / |T| */
    double rel_err_bound; /* a-priori relative error bound of p, first order in the unit
                             roundoffs: 16 (n u + k u_c) R (1 + quad), u of the term
                             precision, k the elimination steps that formed Sigma_C
                             (no-click conditioning steps, or the m sweeps of a state's
                             inverse for its full patterns; 0 for a marginal pattern)
                             with unit roundoff u_c, R = cancel_ratio, quad the
                             largest mean exponent (displaced states; else 0) */
    double log_pvac_n;    /* log P_vac(N) */
    int32_t n_clicks;     /* |C| */
    int32_t prec_used;    /* TOR_PREC_F64, TOR_PREC_DD or TOR_PREC_QD */
    int32_t status;       /* per-result status (TOR_OK or TOR_WARN_PRECISION) */
    int32_t reserved;
} tor_result;

/* Per-context cumulative kernel statistics (HIP events on the context's
 * stream; recorded only while timing is enabled). */
typedef struct {
    double wave_ms;       /* total time of the wave-tier kernel launches */
    double expand_ms;     /* total time of the HBM-tier expansion launches */
    double reduce_ms;     /* total time of the reduction launches */
    int64_t wave_launches;
    int64_t expand_launches;
    int64_t reduce_launches;
    double subsets;       /* number of subset terms evaluated (2^n per sum) */
    int64_t condition_launches; /* launches of no-click conditioning (one per mode, or two per
                                   block of TOR_OPT_COND_BLOCK modes) */
    int64_t fused_launches; /* single-launch subset sums (TOR_OPT_FUSED); each also counts as a
                               wave launch and its time as wave_ms */
} tor_stats;

/* Most wave-tier tasks of a group of subset sums in the single-launch path
 * (TOR_OPT_FUSED); larger groups take the launch chain, whose shared HBM
 * levels then cost less than each unit's own walk from Sigma_C. */
#define TOR_FUSED_MAX_TASKS 4096

/* Options settable on a context (tor_ctx_set_option). */
typedef enum {
    TOR_OPT_TIMING = 0,     /* 1: record HIP events around every launch (default 0) */
    TOR_OPT_TASK_MODES = 1, /* modes per wave-tier task, 1..11, both precisions
                             (default 10 for dd terms, 11 for binary64 terms, or the
                             tuning table's choice per n); setting it clears the
                             table's task sizes */
    TOR_OPT_WAVE_GRID = 2,  /* cap on wave-tier workgroups per launch (default 65536) */
    TOR_OPT_MEM_BUDGET = 3, /* device bytes the context may hold (default 64 GiB) */
    TOR_OPT_ASYNC_POOL = 4, /* tree pool bytes of tor_batch_async (default 4 GiB) */
    TOR_OPT_CHAIN_CLICKS = 5, /* most clicks a chain without postselection may carry,
                              1..TOR_CHAIN_CLICKS (default 15; above 15 the sampler
                              kernel uses more LDS per chain) */
    TOR_OPT_COND_BLOCK = 6,  /* no-click modes conditioned per pair of launches, 1..16
                              (default 16; 1: one launch per mode).  Every value gives
                              bitwise the same result: each entry takes the same
                              rank-2 updates in the same order (Eq. MatrixUpdate
                              iterated over the no-click modes, Sec. II) */
    TOR_OPT_FUSED = 7,       /* 1 (default): a group of zero-mean subset sums whose trees have at
                              most 22 modes and which has at most TOR_FUSED_MAX_TASKS wave-tier tasks runs in
                              one launch (each workgroup rebuilds its unit's node from Sigma_C;
                              block completion counters order the reduction); 0: always the
                              launch chain (one expansion launch per HBM level, the wave tier,
                              the reduction stages).  Both give bitwise the same results: the
                              same nodes, tasks and summation order */
    TOR_OPT_CHAIN_PREC = 8   /* term precision of the chains of gbs_sample, gbs_trace and their
                              displaced and step-traced forms: TOR_PREC_F64 (default; binary64
                              K_j and subset terms, double-double sums) or TOR_PREC_DD
                              (K_j as double-double words, double-double terms; about 2.2x
                              the time).  The persistent loop's chains stay binary64 */
} tor_option;

/* Create a context on HIP device `device` (its own stream, default priority).
 * *out receives the context.  Errors: TOR_EINVAL, TOR_EDEVICE, TOR_ENOMEM. */
tor_status tor_ctx_create(int device, tor_ctx **out);
void tor_ctx_destroy(tor_ctx *ctx);

/* Run the context's work on `stream` (a hipStream_t of the context's device,
 * e.g. a torch stream's handle); NULL restores the context's own stream. */
tor_status tor_ctx_set_stream(tor_ctx *ctx, void *stream);
tor_status tor_ctx_set_option(tor_ctx *ctx, tor_option opt, int64_t value);
tor_status tor_ctx_get_stats(const tor_ctx *ctx, tor_stats *out);
tor_status tor_ctx_reset_stats(tor_ctx *ctx);

/* Autotuner: for each tree size n in [n_lo, n_hi] time the candidate
 * wave-tier task sizes (6..11 modes per task) on a synthetic SPD matrix and
 * keep the fastest for (prec, n) in ctx; with cache_path != NULL also write
 * the context's table as JSON ({"arch": ..., "task_modes": {"dd:24": 9, ...},
 * "persistent_unit_levels": {"pst:24": 2, ...}}).  The choice depends only on
 * (prec, n): results of a query never depend on the other queries it is
 * batched with.  prec must be TOR_PREC_F64 or TOR_PREC_DD.  A context loads
 * the table named by the environment variable TOR_TUNE_CACHE when it is set
 * (an empty value: no table), else the table tor_tuning.json beside the
 * library when it exists. */
tor_status tor_autotune(tor_ctx *ctx, tor_prec prec, int32_t n_lo, int32_t n_hi, const char *cache_path);
tor_status tor_load_tuning(tor_ctx *ctx, const char *cache_path);
/* The task size a tree of n modes will use with precision prec. */
tor_status tor_get_tuning(const tor_ctx *ctx, tor_prec prec, int32_t n, int32_t *task_modes);

/* Thread-local message of the last error on this thread ("" if none). */
const char *tor_last_error(void);

/* Probability of one click pattern of the zero-mean Gaussian state `cov`
 * (m modes).  Sec. II of the paper (signed sum of Eq. (prob) vacuum terms;
 * no-click modes conditioned with Eq. MatrixUpdate).  tol is the relative
 * error target for TOR_PREC_AUTO and for the TOR_WARN_PRECISION flag.
 * Errors: TOR_EINVAL, TOR_ENOTPD, TOR_ETOOBIG, TOR_ENOMEM, TOR_EDEVICE. */
tor_status tor_probability(tor_ctx *ctx, const double *cov, int32_t m, const int8_t *pattern, tor_prec prec,
                           double tol, tor_result *out);

/* Probability of one click pattern of a displaced Gaussian state: covariance
 * cov as for tor_probability and mean vector mean (2m doubles, host, the same
 * interleaved (x_k, p_k) order and hbar = 1 units, so vacuum has cov = I/2).
 * Sec. II of the paper for non-zero means: every vacuum probability of
 * Eq. (prob) carries its mean overlap, det(sigma_Q[A])^{-1/2}
 * exp(-mu_A^T sigma_Q[A]^-1 mu_A / 2), and the no-click conditioning moves
 * the mean with the covariance (the update of the mean beside
 * Eq. MatrixUpdate).  The factor 1/2 in the exponent is the reading of the
 * printed exponent (given for hbar = 2 without it) that reproduces the
 * coherent-state closed form p(click) = 1 - exp(-|alpha|^2).  Fields of out as
 * for tor_probability, except: T is the subset sum with the mean factors of
 * the conditioned state, tor = det(Sigma_C)^{1/2} * T, and rel_err_bound
 * carries a further factor (1 + mu_C^T Sigma_C^-1 mu_C) for the rounding of
 * the exponents.  A zero mean gives the zero-mean result.  prec as for
 * tor_probability, TOR_PREC_QD included (the overlap factors then come from
 * a quad-double exp).  Errors as for tor_probability (TOR_EINVAL also for a
 * NULL or non-finite mean entry of an observed mode). */
tor_status tor_probability_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                     const int8_t *pattern, tor_prec prec, double tol, tor_result *out);

/* The subset sum alone for a given SPD matrix Sigma (2n x 2n row-major,
 * interleaved, host): T = sum_{Y subset of [n]} (-1)^{|Y|} det(Sigma[Y])^{-1/2}.
 * sigma_lo may be NULL; otherwise Sigma = sigma_hi + sigma_lo entrywise
 * (double-double input).  out->p = T, out->log_pvac_n = 0.  n <= 32. */
tor_status tor_subset_sum(tor_ctx *ctx, const double *sigma_hi, const double *sigma_lo, int32_t n, tor_prec prec,
                          double tol, tor_result *out);

/* A state: validated covariance kept on the host (and sigma_Q formed once)
 * for many queries.  cov as above. */
tor_status tor_state_create(tor_ctx *ctx, const double *cov, int32_t m, tor_state **out);
/* A displaced state: cov as above and mean (host, 2m doubles, all finite,
 * as for tor_probability_displaced).  tor_batch and the server evaluate its
 * queries as tor_probability_displaced does (bitwise the same results), and
 * tor_batch_async as tor_batch does; quad-double terms reject it with
 * TOR_EINVAL. */
tor_status tor_state_create_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                      tor_state **out);
void tor_state_destroy(tor_state *st);

/* Per-state preprocessing for full patterns (every mode 1 or 0; Sec. II's
 * vacuum conditioning done once per state instead of once per query).
 * Forms K = sigma_Q^-1 of a state on the GPU by one symmetric 2x2
 * sweep per mode, with det(sigma_Q)^-1/2, in double-double words (prec
 * TOR_PREC_F64, TOR_PREC_DD or TOR_PREC_AUTO) or quad-double words
 * (TOR_PREC_QD), and keeps them with the state (E(m) = m(2m+1) words on the
 * host; the device buffer is freed before returning).  Afterwards tor_batch
 * and the server evaluate a full pattern with at least one no-click mode of
 * this state from G = K[C] (the clicked modes' block) by Jacobi's
 * complementary-minor identity:
 *   p(C, N) = (-1)^n det(sigma_Q)^-1/2 T(G),   T(Sigma_C) = (-1)^n det(G)^1/2 T(G),
 * a gather and one subset tree per query (tor_batch_async takes such full
 * patterns too).  The terms of T(G) are those of
 * T(Sigma_C) times one constant, so the cancellation ratio and error bound
 * are the same.  A double-double inverse serves binary64 and double-double
 * terms (quad-double queries of the state keep the per-query conditioning);
 * a quad-double inverse serves every precision.  Patterns with unobserved
 * modes (-1) keep the per-query conditioning.  A displaced state also keeps
 * h = K mu and mu^T K mu (double-double); its full patterns are the
 * information-form sums of [0, h_C; h_C, G] (each pivot's factor carries
 * exp(+|w|^2/2)): p = (-1)^n det(sigma_Q)^-1/2 exp(-mu^T K mu / 2) T_h(G),
 * in tor_batch, the server and tor_batch_async; quad-double terms
 * take this route from a quad-double inverse (h then in quad-double too),
 * else the per-query conditioning.  Errors:
 * TOR_EINVAL (NULL, bad prec), TOR_ETOOBIG (m > 2048), TOR_ENOMEM,
 * TOR_ENOTPD (a non-positive pivot; a previous inverse is kept).  Not
 * thread-safe against other calls on the state (call it before submitting
 * queries of the state). */
tor_status tor_state_invert(tor_state *st, tor_prec prec);

/* nq queries on one state, patterns = nq x m int8 (row per query), results in
 * out[nq].  All queries' subset trees are evaluated in shared launches, each
 * with its own fixed reduction order, so every result is bitwise identical to
 * the same query run alone.  Per-query failures are reported in
 * out[i].status; the call returns the first error, or TOR_OK /
 * TOR_WARN_PRECISION. */
tor_status tor_batch(tor_ctx *ctx, const tor_state *st, int32_t nq, const int8_t *patterns, tor_prec prec,
                     double tol, tor_result *out);

/* tor_batch for a displaced state: the state's covariance with the mean
 * vector mean (host, 2m doubles, as for tor_probability_displaced) shared by
 * all nq queries.  Zero-mean and displaced trees never share a launch; every
 * result is bitwise that of tor_probability_displaced on the same query.
 * Errors as for tor_batch (TOR_EINVAL also for a NULL mean; a non-finite
 * mean entry of an observed mode fails that query with TOR_EINVAL). */
tor_status tor_batch_displaced(tor_ctx *ctx, const tor_state *st, const double *mean, int32_t nq,
                               const int8_t *patterns, tor_prec prec, double tol, tor_result *out);

/* Stream-ordered form of tor_batch for callers whose patterns and results
 * live in device memory (e.g. torch tensors): d_patterns (nq x m int8, row
 * per query) and d_out (nq tor_result) are device pointers owned by the
 * caller.  The call only enqueues work on `stream` (a hipStream_t; NULL: the
 * context's stream) and returns without waiting; d_patterns is read and
 * d_out written when the stream reaches the call, so both must stay valid
 * until then.  The plan is made on the device for the same trees and
 * reduction order as tor_batch: results (p, p_lo, T, T_lo, abs_sum) are
 * bitwise those of tor_batch; log_p and tor may differ in the last bit.
 * Marginal patterns (entries 1 or -1), and full patterns (entries 1 or 0)
 * of a state inverted by tor_state_invert: G = sigma_Q^-1 over C is
 * gathered on the device and p = (-1)^n det(sigma_Q)^-1/2 T(G) is bitwise
 * tor_batch's; the reported T, abs_sum, cancel_ratio, rel_err_bound and tor
 * of such a query are rescaled to Sigma_C with a binary64 det(G)^1/2 (relative
 * difference from tor_batch's ~1e-15).  On an inverted displaced state the
 * full patterns are the information-form trees of [0, h_C; h_C, G] (p as in
 * tor_state_invert, bitwise tor_batch's) and its marginal patterns the
 * displaced trees, both kinds in one call.  Any other query with a no-click mode
 * (0), or with a bad entry, gets status TOR_EINVAL in its result (per-query
 * conditioning needs host planning: use tor_batch), more than 32 clicks
 * TOR_ETOOBIG.
 * prec: TOR_PREC_F64 or TOR_PREC_DD; TOR_PREC_AUTO is run as TOR_PREC_DD (a
 * query cannot be repeated without a host decision).  Device memory: a
 * workspace whose tree pool holds TOR_OPT_ASYNC_POOL bytes (default 4 GiB);
 * queries are admitted in order while the trees up to them fit, later ones
 * get TOR_ENOMEM.  The first call on a state copies its covariance (and the
 * mean of a displaced state, or the inverse (and h) of an inverted state) to the
 * device (synchronously, once).  The workspace belongs to the context: calls
 * on one context must be ordered (same stream, or the caller waits).
 * Returns TOR_OK once enqueued; argument errors (NULL pointers, nq < 0, bad
 * prec, state of another context) and launch or allocation failures are
 * returned directly. */
tor_status tor_batch_async(tor_ctx *ctx, const tor_state *st, int32_t nq, const int8_t *d_patterns, tor_prec prec,
                           double tol, tor_result *d_out, void *stream);

/* Allocation-free form of tor_batch_async, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It calls no hipMalloc, hipFree or other allocating
 * routine: its whole workspace (plan tables and tree pool) is one static
 * device array of TOR_NOALLOC_SCRATCH_BYTES per GPU, resolved when a context
 * is created on that GPU and held until the process ends.
 *   d_cov       device pointer, 2m x 2m row-major binary64, the zero-mean
 *               covariance (conventions as for cov above), owned by the
 *               caller; it is not validated on the host (finite and
 *               symmetric is the caller's guarantee; a Sigma_C that is not
 *               positive definite gives TOR_ENOTPD in its result)
 *   d_patterns  device, nq x m int8, marginal patterns (1 = click, -1 =
 *               unobserved); a query with a no-click mode (0) or a bad entry
 *               gets TOR_EINVAL in its result, more than 32 clicks TOR_ETOOBIG
 *   d_out       device, nq tor_result records
 *   nq          at most TOR_NOALLOC_MAX_QUERIES
 * prec, tol and stream as for tor_batch_async; the call only enqueues work.
 * The trees share the workspace's tree pool (about 90 MiB of double-double
 * scalars: one double-double tree of n = 24, or many smaller ones); queries
 * are admitted in order while their trees fit, later ones get TOR_ENOMEM in
 * their result.  Results of admitted queries are bitwise those of
 * tor_batch_async on a zero-mean state with the same covariance (same
 * kernels, trees and reduction order).  Every call on a GPU shares that GPU's
 * workspace and leaves its contents behind (each call's plan rewrites what it
 * reads): calls whose work overlaps on one GPU (different streams, or other
 * threads) race, so order them on one stream or wait in between.
 * Errors: TOR_EINVAL (NULL pointer, m <= 0, nq < 0, bad prec), TOR_ETOOBIG
 * (nq above the limit, m too large), TOR_EDEVICE (no workspace address for
 * the device, launch failure). */
#define TOR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
#define TOR_NOALLOC_MAX_QUERIES 4096
tor_status tor_batch_async_noalloc(tor_ctx *ctx, const double *d_cov, int32_t m, int32_t nq,
                                   const int8_t *d_patterns, tor_prec prec, double tol, tor_result *d_out,
                                   void *stream);

/* ------------------------------------------------------------------------
 * Exact chain-rule sampling (the paper's mode-by-mode sampler, Sec. II: each
 * mode's coin is flipped with the conditional no-click probability given the
 * outcomes so far; here that probability is a ratio of two subset sums).
 * ------------------------------------------------------------------------ */

typedef struct {
    int64_t chains_started;   /* chains consumed to produce the samples (deterministic) */
    int64_t chains_accepted;  /* = samples produced */
    int64_t chains_evaluated; /* chains the GPU ran (whole launches) */
    int64_t chains_capped;    /* chains stopped because the clicks exceeded the cap (TOR_OPT_CHAIN_CLICKS) */
    double seconds;           /* wall time of the call */
    double subsets;           /* subset terms evaluated over the consumed chains */
} gbs_stats;

#define TOR_CHAIN_CLICKS 20   /* largest click count a chain may carry */

/* Draw n_samples threshold-detector samples of the zero-mean Gaussian state
 * `cov` (m modes, conventions above).  Modes are measured in ascending order;
 * chain c draws its coin at mode j from Philox4x32-10 with key = seed and
 * counter (c, j), so the output depends only on (cov, n_post, seed).  With
 * n_post >= 0 only chains with exactly n_post clicks are accepted (exact
 * rejection with early stopping: the accepted samples follow the
 * distribution conditioned on n_post clicks); with n_post < 0 every chain
 * with at most TOR_OPT_CHAIN_CLICKS clicks is accepted and longer chains are
 * dropped (counted in chains_capped: the samples then follow the distribution
 * conditioned on at most that many clicks).  Samples are the first accepted
 * chains in chain order.
 * samples: host, n_samples x m bytes (0/1).  stats may be NULL.
 * Per-mode probabilities use binary64 matrices (K_j = sigma_Q[0..j]^-1 formed
 * in double-double and rounded once) and double-double sums.
 * Errors: TOR_EINVAL, TOR_ETOOBIG (n_post > TOR_CHAIN_CLICKS or m > 1024),
 * TOR_EAGAIN (no sample after 2^31 chains), TOR_ENOMEM, TOR_EDEVICE. */
tor_status gbs_sample(tor_ctx *ctx, const double *cov, int32_t m, int32_t n_post, uint64_t seed,
                      int32_t n_samples, uint8_t *samples, gbs_stats *stats);

/* Replay chains chain_begin .. chain_begin + nchains - 1 of gbs_sample with
 * the same (cov, n_post, seed) and report, per chain and mode, the click
 * probability used (NaN after the chain stopped), the uniform draw and the
 * outcome, and per chain its status (1 accepted, 0 rejected, 2 capped).  Any
 * output pointer may be NULL.  Arrays are host, nchains x m (row per chain).
 * A chain is resumable from (seed, chain index): the coins are a pure
 * function of the counter. */
tor_status gbs_trace(tor_ctx *ctx, const double *cov, int32_t m, int32_t n_post, uint64_t seed,
                     int64_t chain_begin, int32_t nchains, double *p_click, double *uniform, uint8_t *outcome,
                     int8_t *status);

/* gbs_sample and gbs_trace for a displaced Gaussian state: mean (host, 2m
 * doubles, interleaved, hbar = 1, all finite) as for
 * tor_probability_displaced.  The paper's sampling rule with non-zero means
 * (Sec. II): each step's click probability is the ratio of two displaced
 * vacuum sums, evaluated in the information form of the measured modes
 * (K_j = sigma_Q[0..j]^-1 and h_j = K_j mu[0..j], double-double, rounded
 * once), where every vacuum probability becomes a common factor times
 * det(K[Z])^-1/2 exp(+h_Z^T K[Z]^-1 h_Z / 2) over the complementary set Z.
 * Chains, coins, postselection and outputs as for the zero-mean calls; a
 * zero mean gives the zero-mean results.  Errors as for gbs_sample /
 * gbs_trace, TOR_EINVAL also for a NULL or non-finite mean. */
tor_status gbs_sample_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                                uint64_t seed, int32_t n_samples, uint8_t *samples, gbs_stats *stats);
tor_status gbs_trace_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                               uint64_t seed, int64_t chain_begin, int32_t nchains, double *p_click,
                               double *uniform, uint8_t *outcome, int8_t *status);

/* gbs_trace (mean == NULL) or gbs_trace_displaced with two more per-step
 * outputs (host, nchains x m, NaN where a step was not evaluated; either may be
 * NULL): cancel_ratio receives max(A0 / |X0|, A1 / |X1|) of the step's split
 * subset sum (X0, X1 the no-click and the all-observed sums whose ratio is
 * P(no click), A0, A1 the sums of their terms' magnitudes; Sec. II), and
 * err_bound an a-priori bound on the absolute error of the step's P(click):
 * 16 ((k + 1) u + u_K) (A0 / |X0| + A1 / |X1|) X0 / X1 + 2^-52 (X0 / X1 +
 * P(click)), k the clicks so far plus one, u the unit roundoff of the terms
 * (2^-53, or 2^-104 with TOR_OPT_CHAIN_PREC = TOR_PREC_DD), u_K = 2m 2^-104
 * for double-double K_j (0 for binary64 K_j, whose rounding the k + 1
 * covers).  A coin u with |u - P(click)| above the bound is decided
 * correctly.  Errors as for gbs_trace. */
tor_status gbs_trace_steps(tor_ctx *ctx, const double *cov, const double *mean, int32_t m, int32_t n_post,
                           uint64_t seed, int64_t chain_begin, int32_t nchains, double *p_click, double *uniform,
                           uint8_t *outcome, int8_t *status, double *cancel_ratio, double *err_bound);

/* The paper's benchmark mode (Sec. III, "Runtime"): one sample whose
 * outcomes are fixed in advance, measured mode by mode from the last mode down
 * (Sec. II).  outcomes[m] (host) holds 1 = click, 0 = no click, -1 = not
 * measured (traced out).  step_p[j] (host, m doubles, may be NULL) receives
 * P(outcome of mode j | outcomes of the modes measured before it), 1 for
 * unmeasured modes; *total the probability of the whole pattern (the product
 * of the steps), with rel_err_bound the largest bound of the step sums and
 * cancel_ratio the largest cancellation ratio met.
 * Each no-click step conditions the matrix of the remaining observed modes on
 * the measured mode (one GPU step, Eq. MatrixUpdate); the step probabilities
 * are ratios of the subset sums over the clicks so far before and after each
 * step, all of them evaluated in one batched launch.  Clicks <= 32, observed
 * modes <= 1024.  prec as for tor_probability (AUTO repeats in double-double
 * the sums whose binary64 bound exceeds tol); TOR_PREC_QD conditions and sums
 * in quad-double (one tree per step: slower, for chains whose double-double
 * bound exceeds tol, e.g. the worst case with 20 clicks on 800 modes).
 * Errors: TOR_EINVAL, TOR_ETOOBIG, TOR_ENOTPD, TOR_ENOMEM, TOR_EDEVICE;
 * TOR_WARN_PRECISION when the bound exceeds tol. */
tor_status gbs_chain_fixed(tor_ctx *ctx, const double *cov, int32_t m, const int8_t *outcomes, tor_prec prec,
                           double tol, double *step_p, tor_result *total);

/* gbs_chain_fixed for a displaced state (the paper's mode-by-mode rule with
 * non-zero means, Sec. II): mean (host, 2m doubles, interleaved, hbar = 1) as
 * for tor_probability_displaced.  Each no-click step also moves the mean of
 * the remaining modes, and every vacuum probability carries its mean-overlap
 * factor; rel_err_bound includes the exponent factor (1 + mu^T Sigma^-1 mu)
 * of each step's sum.  prec as for gbs_chain_fixed (TOR_PREC_QD included).
 * Errors as for gbs_chain_fixed, TOR_EINVAL also for a NULL mean or a
 * non-finite mean entry of a measured mode. */
tor_status gbs_chain_fixed_displaced(tor_ctx *ctx, const double *cov, const double *mean, int32_t m,
                                     const int8_t *outcomes, tor_prec prec, double tol, double *step_p,
                                     tor_result *total);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of probability queries.
 *
 * Each worker owns a stream and device buffers.  A free worker takes the
 * oldest pending queries that fit its memory budget (at most max_batch) and
 * evaluates them as one fused batch (see tor_batch); queries submitted while
 * batches are on the GPU are admitted into the next free worker's batch, so
 * the batches of different workers overlap on the device.  Every result is
 * bitwise identical to the same query evaluated alone.  Thread-safe: any
 * thread may submit, poll or wait.
 * ------------------------------------------------------------------------ */

typedef struct tor_server tor_server;

typedef struct {
    int32_t workers;         /* concurrent batches (each its own stream); default 2, at most 16 */
    int32_t max_pending;     /* admission: queries waiting; further submits get TOR_EAGAIN (default 65536) */
    size_t mem_budget_bytes; /* device bytes per batch (admission by memory; default 16 GiB) */
    tor_prec prec;           /* precision policy of every query (TOR_PREC_DD recommended; with
                                TOR_PREC_QD each worker evaluates one query at a time through
                                the quad-double single-query path, bitwise its result) */
    double tol;              /* relative error target; <= 0 means 1e-10 */
    int32_t max_batch;       /* queries per fused batch (default 4096) */
} tor_server_opts;

typedef struct {
    int64_t submitted;
    int64_t completed;
    int64_t batches;
    int64_t max_batch_seen;
    int64_t pending;
} tor_server_stats;

/* Start a server on ctx's device (opts may be NULL for defaults).  The server
 * must be stopped before ctx is destroyed. */
tor_status tor_server_start(tor_ctx *ctx, const tor_server_opts *opts, tor_server **out);
/* Queue one query on state st (st must outlive the query).  The pattern is
 * reduced to its conditioned matrix before returning.  *ticket identifies the
 * result.  TOR_EAGAIN: not admitted (queue full); other errors as
 * tor_probability. */
tor_status tor_submit(tor_server *srv, const tor_state *st, const int8_t *pattern, uint64_t *ticket);
/* TOR_EAGAIN while the query is pending; otherwise fills *out (and the
 * submit-to-completion latency in seconds, if latency_s is not NULL), releases
 * the ticket and returns the result's status. */
tor_status tor_poll(tor_server *srv, uint64_t ticket, tor_result *out, double *latency_s);
/* As tor_poll but blocks until the result is ready. */
tor_status tor_wait(tor_server *srv, uint64_t ticket, tor_result *out, double *latency_s);
tor_status tor_server_get_stats(tor_server *srv, tor_server_stats *out);
/* Finish every pending query, then stop the workers and free the server. */
tor_status tor_server_stop(tor_server *srv);

/* ------------------------------------------------------------------------
 * Persistent request loop: one long-running kernel on the device takes the
 * work of probability queries and of sampling batches as they are submitted.
 *
 * Requests go, in submission order, into a ring of TOR_PS_SLOTS request slots
 * in host-coherent memory.  The kernel's workgroups claim the work units of
 * the published requests with atomic counters on the device (a probability
 * query of n clicks: 2^g subtrees of its subset tree, the schedule (task
 * modes, depth-first levels per unit) per n from the context's tuning table;
 * a sampling batch: one chain per unit), so the units of a request that
 * arrives while others are on the GPU start as soon as workgroups free up,
 * and the work of different requests overlaps on the device.  The last unit
 * of a request sums its partial results and sets the request's completion
 * word (a system-scope release the host reads).  No unit waits for another;
 * a workgroup waits only for new work.  The kernel exits on the stop flag, or
 * as a whole once every workgroup has been idle_ms without work (workgroups
 * never leave one by one, so a long request with few units does not shrink
 * the kernel), and is launched again on demand (by submit and poll).
 *
 * Probability queries (Sec. II of the paper, as tor_probability): zero-mean
 * states, marginal patterns (1 and -1 entries) and full patterns (1 and 0
 * entries) of a state inverted by tor_state_invert; double-double terms.
 * Every result is bitwise that of tor_batch on the same state and pattern
 * with TOR_PREC_DD (same trees, tasks and reduction order), whatever else is
 * in flight.  Sampling batches: chains chain_begin .. chain_begin + nchains - 1
 * of gbs_sample / gbs_trace with the same (state, n_post, seed): the outcomes
 * and statuses are bitwise gbs_trace's (binary64 terms); at most
 * TOR_PS_CHAIN_CLICKS clicks per chain (n_post, and the cap of chains
 * without postselection).
 * Admission: a request is refused with TOR_EAGAIN when its ring slot is still
 * held (poll results promptly: a slot is freed when its result is read), when
 * its partial sums do not fit mem_budget_bytes of device memory (2^(n - J)
 * task partials of 32 bytes), or when a batch's outputs do not fit the pinned
 * chain buffer.  Thread-safe.  While the kernel runs it holds every CU it
 * fits, so other work on the device waits for its idle exit.
 * ------------------------------------------------------------------------ */

#define TOR_PS_SLOTS 4096
#define TOR_PS_CHAIN_CLICKS 15

typedef struct tor_pserver tor_pserver;

typedef struct {
    double tol;                /* relative error target of the results' status; <= 0: 1e-10 */
    size_t mem_budget_bytes;   /* device bytes for the partial sums of requests in flight (default 1 GiB) */
    size_t chain_buffer_bytes; /* pinned host bytes for the outputs of sampling batches (default 64 MiB) */
    int32_t grid;              /* workgroups of the kernel; 0: as many as fit the device at once */
    int32_t idle_ms;           /* the kernel exits once all its workgroups are this long without work (default 50) */
} tor_pserver_opts;

typedef struct {
    int64_t submitted;
    int64_t completed;
    int64_t pending;   /* submitted and not yet read */
    int64_t units;     /* work units published */
    int64_t launches;  /* launches of the persistent kernel */
    int64_t device_cursor;    /* index of the request whose units the kernel is claiming */
    int64_t device_published; /* requests the kernel has seen published */
    int32_t running;   /* 1 while the kernel runs */
    int32_t workgroups;          /* workgroups per launch */
    int32_t workgroups_started;  /* workgroups started over all launches */
    int32_t workgroups_peak;     /* most workgroups resident at once */
} tor_pserver_stats;

/* Start the loop on ctx's device (opts may be NULL) and launch its kernel.
 * The server must be stopped before ctx or any state it serves is destroyed.
 * Errors: TOR_EINVAL, TOR_ENOMEM, TOR_EDEVICE. */
tor_status tor_pserver_start(tor_ctx *ctx, const tor_pserver_opts *opts, tor_pserver **out);
/* Submit a probability query of state st (pattern as for tor_probability);
 * *ticket names its result.  Errors: TOR_EINVAL (a displaced state, a pattern
 * with no-click modes that is not a full pattern of an inverted state, a bad
 * entry), TOR_ETOOBIG (more than 32 clicks), TOR_ENOTPD, TOR_EAGAIN (not
 * admitted: try again after reading results). */
tor_status tor_pserver_submit(tor_pserver *srv, const tor_state *st, const int8_t *pattern, uint64_t *ticket);
/* Submit a sampling batch: chains chain_begin .. chain_begin + nchains - 1 of
 * gbs_sample with postselection n_post (< 0: none) and seed on state st.
 * Errors: TOR_EINVAL, TOR_ETOOBIG (n_post > TOR_PS_CHAIN_CLICKS, m > 1024),
 * TOR_ENOTPD, TOR_ENOMEM, TOR_EAGAIN. */
tor_status tor_pserver_submit_chains(tor_pserver *srv, const tor_state *st, int32_t n_post, uint64_t seed,
                                     int64_t chain_begin, int32_t nchains, uint64_t *ticket);
/* Result of a probability query: TOR_EAGAIN while pending (with wait != 0,
 * block until ready); else fills *out (and the submit-to-result latency in
 * seconds), frees the ticket and returns the result's status. */
tor_status tor_pserver_poll(tor_pserver *srv, uint64_t ticket, int32_t wait, tor_result *out, double *latency_s);
/* Result of a sampling batch: outcomes (host, nchains x m bytes 0/1) and
 * status (host, nchains: 1 accepted, 0 rejected, 2 capped) as gbs_trace
 * reports them; either may be NULL.  TOR_EAGAIN while pending (wait as for
 * tor_pserver_poll). */
tor_status tor_pserver_poll_chains(tor_pserver *srv, uint64_t ticket, int32_t wait, uint8_t *outcomes,
                                   int8_t *status, double *latency_s);
tor_status tor_pserver_get_stats(tor_pserver *srv, tor_pserver_stats *out);
/* Autotuner of the persistent schedule: for each tree size n in [n_lo, n_hi]
 * and every depth-first unit depth t (units of 2^t wave tasks; the task size
 * is the batched path's, so results stay bitwise tor_batch's) time one query
 * alone and a burst of 32 (a synthetic 32-mode state), and keep in the
 * server's context the t of the least time per query in the burst among those
 * whose time alone is within 1.5x (+ 20 us) of the least;
 * with cache_path also write the context's whole table (task sizes and unit
 * depths) as JSON for tor_load_tuning.  With the environment variable
 * TOR_TUNE_VERBOSE set (not "0") every measurement goes to stderr.  A context
 * loads TOR_TUNE_CACHE when that variable is set, else the table
 * tor_tuning.json beside the library when it exists. */
tor_status tor_pserver_autotune(tor_pserver *srv, int32_t n_lo, int32_t n_hi, const char *cache_path);
/* Finish every submitted request (unread results are dropped), set the stop
 * flag, wait for the kernel to exit and free the server. */
tor_status tor_pserver_stop(tor_pserver *srv);

#ifdef __cplusplus
}
#endif

#endif /* TOR_H */
