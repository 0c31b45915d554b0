/*
 * bt.h -- C ABI of libbt: expected values over the Bernoulli paths of a
 * recombinant binomial tree on one AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Popuri, Raim, Neerchal, Gobbert, "Parallelizing
 * Computation of Expected Values in Recombinant Binomial Trees"):
 *   An N-step tree moves the price S up by u with probability p or down by
 *   d = 1/u (Section 2, assumptions A1-A3).  A path is x in {0,1}^N, x_t = 1
 *   an up move; S_t(x) = S u^(2 U_t - t) with U_t the ups among the first t
 *   steps.  The value of a path-dependent payoff f is the discounted
 *   expectation over all 2^N paths,
 *       V = e^{-rT} sum_x p^{U_N}(1-p)^{N-U_N} f(S_1(x), ..., S_N(x)),
 *   eq. (f13) (eq. (expval) discounted).  The paper writes the interest rate
 *   q; here it is r.  Paths are numbered with the first step as the most
 *   significant bit (Section 3: the rank bits lead the path).
 *
 * Conventions for every function:
 *   - Return 0 (BT_OK) or a negative BT_E* code; nothing throws across the
 *     ABI.  bt_strerror() names a code.
 *   - Host pointers (bt_option, bt_result, arrays) are owned by the caller and
 *     only read/written during the call.  Device memory the library needs
 *     (tables, partial sums) is owned by the library: by a plan until
 *     bt_plan_destroy, or by the library's per-device cache of buffers for
 *     the synchronous one-shot calls (kept until the process ends, up to
 *     2 GiB of idle buffers per device) -- or by the caller, for the *_ws
 *     calls, which take a device workspace.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Functions documented as "enqueue" only enqueue work on it;
 *     the others synchronize it before returning.
 *   - Everything runs on the current HIP device of the calling thread.
 */
#ifndef BT_H
#define BT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define BT_OK 0
#define BT_EINVAL (-1)    /* an argument is out of its documented domain   */
#define BT_ERANGE (-2)    /* N (or a split) exceeds what the call supports */
#define BT_ENOMEM (-3)    /* device or host allocation failed / over budget */
#define BT_EDEVICE (-4)   /* a HIP call failed, or no gfx950 device         */
#define BT_EAGAIN (-5)    /* server: result not ready yet                   */
#define BT_ENOTFOUND (-6) /* server: unknown ticket                         */
#define BT_ESHUTDOWN (-7) /* server: stopped                                */

/* ---- payoffs ----------------------------------------------------------
 * All use the window t = 1..N (S_0 excluded), as the paper's Asian and
 * lookback payoffs do (Section 5).  Eqs. (call), (put) of Section 2 for the
 * European pair. */
typedef enum {
    BT_ASIAN_CALL = 0,         /* max(mean(S_1..S_N) - K, 0)                 */
    BT_ASIAN_PUT = 1,          /* max(K - mean(S_1..S_N), 0)   (Section 5)   */
    BT_LOOKBACK_FLOAT = 2,     /* max(S_1..S_N) - S_N  (floating strike)     */
    BT_LOOKBACK_FIXED_PUT = 3, /* max(K - min(S_1..S_N), 0)    (Section 5)   */
    BT_EURO_CALL = 4,          /* max(S_N - K, 0)              eq. (call)    */
    BT_EURO_PUT = 5            /* max(K - S_N, 0)              eq. (put)     */
} bt_payoff;

/* Per-path arithmetic.  BT_FP64: every quantity in FP64.  BT_FP32_KAHAN
 * (exact pricing): per-path payoff arithmetic in FP32 with Kahan-compensated
 * per-lane sums; path weights p^j(1-p)^(N-j), prefix states and every
 * cross-lane reduction stay in FP64.  Monte Carlo calls take the same value
 * under the name BT_FP32: the suffix walk (prices, running sums and
 * extremes, the payoff) runs in FP32, while each lane's sums over its draws
 * and every combination across lanes and strata are FP64, so there is no
 * FP32 sum to compensate. */
typedef enum { BT_FP64 = 0, BT_FP32_KAHAN = 1, BT_FP32 = 1 } bt_precision;

/* Tree parameterisation for bt_params (Section 2). */
typedef enum {
    BT_SCHEME_CRR = 0,   /* u = exp(sigma sqrt(dt))                          */
    BT_SCHEME_SEYDEL = 1 /* u = beta + sqrt(beta^2 - 1), beta = (e^{-r dt} +
                            e^{(r+sigma^2) dt})/2; the paper prints "+1"
                            under the root, read as "-1" (it reproduces the
                            exact values printed in Section 5).              */
} bt_scheme;

/* One option: the paper's problem statement.  S > 0 spot, u > 1 up factor
 * (d = 1/u, A1), 0 < p < 1 up probability (A2), r the rate used for the
 * discount e^{-rT} (A3), T > 0 maturity, K >= 0 strike, N >= 1 steps,
 * payoff a bt_payoff. */
typedef struct {
    double S, u, p, r, T, K;
    int32_t N;
    int32_t payoff;
} bt_option;

/* Result of one pricing call.
 *
 * err_bound: a bound on the rounding error of `value`, computed for every
 * exact result (one-shot, batch, plan, server) from the computation that
 * produced it: |value - V| <= err_bound, where V is the same quantity in
 * exact arithmetic (for exact pricing, eq. (f13) itself).  It is a
 * first-order forward error bound (each FP64 operation within 2^-53 of its
 * result, each FP32 one within 2^-24, library pow/exp within two units in
 * the last place) with a margin of 2^-20 of itself for the second-order
 * terms: the rounding of the stored prefix and suffix operands (FP32
 * records: 2^-24 of each), of the path weights, of every FP32 or FP64 sum
 * that leads to the value.  For the FP32 form of a binomial tree the
 * rounding of the stored operands counts only on the paths that can reach
 * the money (a histogram of the suffix operands against each prefix's
 * threshold, computed on the GPU), so the bound stays within about 7.5e-7
 * |V| however far the option is out of the money, and is exactly 0 when no
 * path can pay.  Typical sizes: FP64 1e-13 |V| (its operand rounding is
 * summed over all paths: deep out-of-the-money options reach 1e-8 |V|);
 * FP32 binomial 6e-7 to 7.5e-7 |V|; FP32 time-varying and trinomial trees,
 * whose weights ride in the FP32 multiplier and whose terms pass a chain of
 * 32 FP32 multiply-adds, 2.5e-6 |V|.  For Monte Carlo estimates the error
 * is statistical and err_bound is the standard error std_err: not a bound
 * (|value - V| exceeds it about one time in three), but the figure that the
 * estimate's own rounding error stays far below. */
typedef struct {
    double value;        /* discounted expected payoff                      */
    double err_bound;    /* exact: rounding-error bound of value; MC:
                            std_err (see above)                             */
    double std_err;      /* MC: sqrt(var_est); exact: 0                     */
    double var_est;      /* MC: plug-in variance estimate of value (the
                            paper's 1/R_m normalisation); exact: 0          */
    double var_unbiased; /* MC: same with 1/(R_m - 1); exact: 0             */
    double var_plain;    /* MC: estimated variance of plain Monte Carlo
                            (eq. (mc2)) with the same number of paths, from
                            the same draws: (sum_z P(D_z) (s_z^2 +
                            thetahat_z^2) - value^2) / paths, discounted (for
                            basic MC, var_est itself); NaN for Shared-Sample
                            estimates; exact: 0                              */
    uint64_t paths;      /* paths evaluated                                 */
    int32_t split;       /* exact: suffix steps k; MC: prefix steps r       */
    int32_t status;      /* BT_OK or an error for this entry (batch/server)  */
} bt_result;

/* Launch shape of the enumeration.  Zero fields mean "choose": the library
 * then uses its autotuned table (bt_autotune) or built-in defaults, both
 * made for throughput over many trees.  One tree of depth 11..31 alone
 * finishes 2-4x sooner with the server's one-tree shapes (listed with
 * bt_server_config), passed here. */
typedef struct {
    int32_t k;        /* suffix steps owned by lanes, 0 or 1..16 (larger than
                         an option's N means N)                              */
    int32_t chunk;    /* prefixes per rectangle, 0 or a multiple of 4 in
                         [4, 2048]                                           */
    int32_t waves;    /* waves per workgroup: 0 or 4                        */
    int32_t grid;     /* workgroups of the enumeration launch; 0 = one per
                         rectangle of paths; fewer make each workgroup take
                         rectangles g, g + grid, ... in turn                 */
} bt_tuning;

/* ---- basics ------------------------------------------------------------ */

/* Name of an error code (static string). */
const char *bt_strerror(int code);

/* Select and check the device (must be gfx950) for the calling thread and
 * set up the library's per-device state.  Optional: every entry point does
 * it on first use on the current device. */
int bt_init(int device);

/* Section 2, A1-A3: u and p from (sigma, r, T, N) with dt = T/N and
 * p = (e^{r dt} - d)/(u - d).  BT_EINVAL if sigma <= 0, T <= 0, N < 1 or the
 * resulting p is not in (0, 1). */
int bt_params(double sigma, double r, double T, int32_t N, int32_t scheme,
              double *u, double *p);

/* ---- exact enumeration (eq. (f13), Section 3) --------------------------
 * Each path x = (z, s) is split into a prefix z of P = N - k steps and a
 * suffix s of k steps (Section 3's rank prefix, here one prefix per step of
 * a work item's loop).  Prefix states are computed once per prefix and
 * suffix states once per suffix; each path then costs one clamped
 * difference and one multiply-add.  Supports 1 <= N <= 40. */

/* Price one option exactly.  tune may be NULL.  Synchronous: the result is
 * in *out when the call returns.  BT_ERANGE if N > 40. */
int bt_price_exact(const bt_option *opt, int32_t precision,
                   const bt_tuning *tune, bt_result *out, void *stream);

/* Time-varying moves (the case named after eq. (f12); eq. (f13) with
 * p(x) = prod_t p_t^{x_t} (1 - p_t)^{1 - x_t}): step t = 1..N multiplies
 * the price by u_t (up) or 1/u_t (down).  u_t[t-1], p_t[t-1] are host
 * arrays of N entries, read during the call; opt->u and opt->p are
 * ignored.  The tree need not recombine.  Prices are products of the step
 * factors along the path.  FP32: the path weight of a prefix is folded
 * into its FP32 factor (no up-count groups exist); BT_ERANGE if the
 * prefix weights span more than 2^100.  BT_EINVAL if some u_t <= 1, is not
 * finite, or p_t is not in (0, 1); BT_ERANGE if N > 40.  Synchronous. */
int bt_price_exact_tv(const bt_option *opt, const double *u_t, const double *p_t,
                      int32_t precision, const bt_tuning *tune, bt_result *out,
                      void *stream);

/* Trinomial trees (Section 3 notes that the path partition applies to trees
 * with more than two branches, citing Boyle's trinomial tree): each step
 * multiplies the price by opt->u (up, probability opt->p), 1 (middle,
 * probability 1 - opt->p - p_down) or 1/opt->u (down, p_down), and eq.
 * (f13) sums over the 3^N paths.  A path is N base-3 digits, first step
 * most significant (0 down, 1 middle, 2 up); the split puts k = min(N, 10)
 * digits (or tune->k, at most 12) in the suffix and at most 16 in the
 * prefix.  FP32: the prefix weight is folded into its FP32 factor, as for
 * time-varying moves.  BT_EINVAL if p_down <= 0 or opt->p + p_down > 1
 * (a zero middle probability is allowed); BT_ERANGE if N > 26, or the
 * split would put more than 16 digits in the prefix or 12 in the suffix,
 * or (FP32) the nonzero prefix weights span more than 2^100.
 * paths = 3^N.  Synchronous. */
int bt_price_exact_trinomial(const bt_option *opt, double p_down, int32_t precision,
                             const bt_tuning *tune, bt_result *out, void *stream);

/* Boyle's trinomial parameters: u = e^{lambda sigma sqrt(dt)} and the up and
 * down probabilities matching the mean e^{r dt} and the variance
 * e^{2 r dt} (e^{sigma^2 dt} - 1) of the step.  BT_EINVAL unless all three
 * probabilities come out positive (lambda too small gives a negative
 * middle probability). */
int bt_params_trinomial(double sigma, double r, double T, int32_t N, double lambda,
                        double *u, double *p_up, double *p_down);

/* Price n options exactly in one enumeration launch (the rectangles of
 * paths of all options in one list, largest first).
 * outs[i] corresponds to opts[i]; per-entry status in outs[i].status.
 * Results are bit-identical to pricing each option alone with the same
 * tuning.  The plan is built in a device buffer from the library's
 * per-device cache of one-shot buffers (allocated on first need, then
 * reused: a repeated call of the same size allocates nothing), and the call
 * synchronizes `stream` once, to return the results. */
int bt_price_batch(const bt_option *opts, int32_t n, int32_t precision,
                   const bt_tuning *tune, bt_result *outs, void *stream);

/* Device bytes the plan of bt_price_batch(opts, n, precision, tune) needs:
 * the workspace size for bt_price_batch_ws / bt_price_exact_ws.  Checks
 * the arguments as bt_plan_create does (same errors); touches no device. */
int bt_plan_bytes(const bt_option *opts, int32_t n, int32_t precision,
                  const bt_tuning *tune, size_t *bytes);

/* bt_price_batch (same arguments, kernels, shapes and results, bit for
 * bit) in caller-owned device memory: d_workspace is ws_bytes of device
 * memory on the current device (for example a torch tensor's storage),
 * 256-byte aligned, at least bt_plan_bytes; the library writes the whole
 * plan there (tables, partial sums, values) and allocates nothing.  The
 * caller keeps ownership; the workspace is in use from the call until it
 * returns (the call synchronizes `stream` once), and its contents are never
 * read before being written.  BT_EINVAL for a NULL or misaligned workspace,
 * BT_ENOMEM if ws_bytes is too small. */
int bt_price_batch_ws(const bt_option *opts, int32_t n, int32_t precision,
                      const bt_tuning *tune, bt_result *outs, void *d_workspace,
                      size_t ws_bytes, void *stream);
/* One option (n = 1) of bt_price_batch_ws. */
int bt_price_exact_ws(const bt_option *opt, int32_t precision, const bt_tuning *tune,
                      bt_result *out, void *d_workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): bt_price_batch with the same arguments,
 * kernels, launch shapes and results (bit for bit), but the plan lives in a
 * fixed 64 MiB array that the library's code object holds on each device
 * from the library's first use there until the process ends; the call
 * allocates no device memory.  BT_ENOMEM if the plan of these options needs
 * more than 64 MiB (a single option fits up to N = 36 in FP64 with the
 * built-in shapes).  Calls on one device are serialized by the library for
 * their whole duration (the call synchronizes `stream` before returning);
 * each call overwrites the array, whose previous contents are never read.
 * Synchronous. */
int bt_price_batch_noalloc(const bt_option *opts, int32_t n, int32_t precision,
                           const bt_tuning *tune, bt_result *outs, void *stream);

/* ---- plans: the same computation, stage by stage ------------------------
 * A plan owns the device tables of n options.  The three enqueue stages are
 * what bt_price_exact / bt_price_batch run; they are exposed so that a
 * caller can time or graph-capture them.  All enqueue calls are
 * asynchronous on `stream`. */
typedef struct bt_plan bt_plan;

int bt_plan_create(const bt_option *opts, int32_t n, int32_t precision,
                   const bt_tuning *tune, bt_plan **plan);

/* A plan for bt_price_exact_trinomial's computation over opts[0..n): each
 * option has its own u and up probability p, all share p_down; one table
 * launch, one enumeration and one reduction serve them all, and each
 * option's value equals its one-option plan's bit for bit.  Same errors as
 * bt_price_exact_trinomial, checked for every option (BT_EINVAL if n < 1). */
int bt_plan_create_trinomial(const bt_option *opts, int32_t n, double p_down,
                             int32_t precision, const bt_tuning *tune, bt_plan **out);

/* A plan for bt_price_exact_tv's computation over opts[0..n), options of one
 * depth N that share the time-varying moves u_t[0..N), p_t[0..N) (their own
 * u and p are ignored; S, K, r, T and the payoff are each option's): the
 * step arrays are copied into the plan's device memory, so the caller may
 * free them on return; each option's value equals its one-option plan's
 * bit for bit.  Same errors as bt_price_exact_tv; BT_EINVAL if n < 1 or
 * the options' N differ. */
int bt_plan_create_tv(const bt_option *opts, int32_t n, const double *u_t, const double *p_t,
                      int32_t precision, const bt_tuning *tune, bt_plan **out);
/* Tree parameters, weights, suffix tables and prefix states (enqueue). */
int bt_plan_tables(bt_plan *plan, void *stream);
/* The enumeration: every path of every option (enqueue). */
int bt_plan_enumerate(bt_plan *plan, void *stream);
/* Deterministic fixed-order reduction of the work-item partials to one
 * discounted value per option, in device memory (enqueue). */
int bt_plan_reduce(bt_plan *plan, void *stream);
/* Copy the values to the host and synchronize `stream`. */
int bt_plan_results(bt_plan *plan, bt_result *outs, void *stream);
/* Device pointer to the n discounted values, followed by their n error
 * bounds (bt_result.err_bound), in the caller's option order (valid until
 * destroy). */
int bt_plan_device_values(bt_plan *plan, double **d_values);
/* Capture tables + enumerate + reduce into a HIP graph owned by the plan;
 * bt_plan_launch_graph replays it on `stream` (enqueue). */
int bt_plan_capture(bt_plan *plan, void *stream);
int bt_plan_launch_graph(bt_plan *plan, void *stream);
/* Number of work items and launch shape actually used. */
int bt_plan_info(const bt_plan *plan, uint64_t *items, bt_tuning *used);
int bt_plan_destroy(bt_plan *plan);

/* Debug export (synchronous) for bit-exact checks of the tables of option
 * `i` of a plan after bt_plan_tables: for every prefix position q in
 * [0, 2^P) the prefix index z (its P steps, first step most significant) and
 * its up-count a; for every suffix s in [0, 2^k) its up-count b.  Arrays are
 * host memory of 2^P and 2^k entries.  FP64 plans store prefix z at
 * position z; FP32 plans store the prefixes ordered by up-count, then z. */
int bt_plan_debug_tables(bt_plan *plan, int32_t i, uint64_t *prefix_z,
                         int32_t *prefix_a, int32_t *suffix_b, void *stream);

/* ---- Partitioned (prefix-stratified) Monte Carlo, Section 4 -------------
 * Strata are the 2^r prefixes of the first r steps, each weighted by its
 * exact probability P(D_z) = p^a (1-p)^(r-a) (eq. (mc9)); each stratum gets
 * R_m suffix draws (equal allocation, the setting of Theorem 1), and
 *   value   = e^{-rT} sum_z P(D_z) thetahat_z                 eq. (mc12)
 *   var_est = e^{-2rT} sum_z P(D_z)^2 s_z^2 / R_m          (eq. (mc13),
 *             first line, with s_z^2 the plug-in (1/R_m) sample variance)
 * Suffix step j (0-based) of sample m in stratum z reads the 16-bit half
 * h_j of word (j%8)/2 of Philox4x32-10(counter = (j/8, m, z, stream_id),
 * key = (seed lo, seed hi)): the high half for even j, the low half for odd
 * j.  With thr = floor(p 2^32) = (thr_hi, thr_lo) in halves, the step goes
 * up iff h_j < thr_hi, and on a tie (h_j == thr_hi) iff g_j < thr_lo, g_j
 * the high half of word 0 of the block with counter (2^31 + j, m, z,
 * stream_id): the step's uniform is the 32-bit (h_j, g_j) and
 * P(up) = thr / 2^32 exactly.  r = 0 is basic Monte Carlo (eq. (mc2)).
 * Requires 0 <= r < N <= 64, r <= 30, 1 <= R_m, 2^r R_m <= 2^40.
 * precision: BT_FP32 (= BT_FP32_KAHAN) walks the suffixes in FP32, BT_FP64
 * in FP64; per-lane sums and the stratum combine are FP64 either way. */
int bt_price_stratified(const bt_option *opt, int32_t prefix_steps,
                        int32_t samples_per_stratum, uint64_t seed,
                        uint32_t stream_id, int32_t precision, bt_result *out,
                        void *stream);

/* Asynchronous form: writes {value, var_est, var_unbiased, var_plain}
 * (4 doubles) to device memory d_out; its scratch comes from HIP's
 * stream-ordered allocator (hipMallocAsync / hipFreeAsync on `stream`). */
int bt_enqueue_stratified(const bt_option *opt, int32_t prefix_steps,
                          int32_t samples_per_stratum, uint64_t seed,
                          uint32_t stream_id, int32_t precision, double *d_out,
                          void *stream);

/* Monte Carlo estimators of Section 4 behind one call.
 *  BT_MC_PARTITIONED:   R_m = `samples` draws in every stratum (as
 *                       bt_price_stratified).
 *  BT_MC_PROPORTIONAL:  `samples` = R in total (R <= 2^30), R_m =
 *                       max(1, round(R P(D_m))) (the allocation the text
 *                       chooses before eq. (mc13); rounding, and at least one
 *                       draw, are this library's reading).  Draws as
 *                       for BT_MC_PARTITIONED.  var_est = e^{-2rT} sum_m
 *                       sum_i (V_mi - thetahat_m)^2 / R^2, the estimator
 *                       printed after eq. (mc13) for this allocation;
 *                       var_unbiased = e^{-2rT} sum_m P(D_m)^2 s_m^2 / R_m
 *                       with s_m^2 over R_m - 1 (NaN if every R_m is 1).
 *  BT_MC_SHARED_SAMPLE: the Remark's estimator, eq. (mc16): R = `samples`
 *                       suffix draws shared by all 2^r prefixes; each draw i
 *                       contributes h_i = sum_z P(D_z) V(z, y_i), evaluated
 *                       over every prefix (2^r R paths); value = e^{-rT} mean
 *                       of h, var_est = e^{-2rT} sum_i (h_i - mean)^2 / R^2
 *                       (the printed estimator, read with the overall mean).
 *                       Draw i is the suffix of sample i in stratum
 *                       0xFFFFFFFF, drawn as for BT_MC_PARTITIONED.
 *                       Requires r <= 26, R <= 2^31 and
 *                       (2^r / chunk) R <= 2^27 (chunk = the prefixes per
 *                       rectangle, up to 2048).
 * Synchronous; `paths` = total paths evaluated. */
typedef enum {
    BT_MC_PARTITIONED = 0,
    BT_MC_PROPORTIONAL = 1,
    BT_MC_SHARED_SAMPLE = 2
} bt_mc_estimator;

int bt_price_mc(const bt_option *opt, int32_t estimator, int32_t prefix_steps,
                uint64_t samples, uint64_t seed, uint32_t stream_id,
                int32_t precision, bt_result *out, void *stream);

/* Debug export: the suffix up/down bits the MC kernel draws for sample m of
 * stratum z (L = N - r bits, first step first), for bit-exact checks. */
int bt_mc_debug_bits(uint64_t seed, uint32_t stream_id, uint32_t z, uint32_t m,
                     int32_t L, double p, int32_t *bits, void *stream);

/* ---- autotuning ---------------------------------------------------------
 * The split k and the chunk size per depth N come from one rule (k near
 * N/2 within [8, 16], chunks of max(cmin, 2^P / div) prefixes); the
 * autotuner times tables + enumeration of a whole batch under each of a
 * set of rules and keeps the fastest in the library's table for the depths
 * concerned (used whenever a bt_tuning field is 0).  Synchronous.  Each
 * candidate is timed in a plan of its own, and only the winner is written
 * to the table (once, at the end): pricing on other threads meanwhile sees
 * the old shapes or the new ones, never a candidate.  BT_EDEVICE (or the
 * first plan error) if no candidate could be timed; the table is then left
 * as it was.
 * bt_autotune: a synthetic batch of Asian calls with depths n_lo..n_hi
 * (about 2^34 paths in all).  BT_EINVAL if the range is outside [1, 40]. */
int bt_autotune(int32_t n_lo, int32_t n_hi, int32_t precision, void *stream);
/* The same search on the caller's own batch (host array of n options, as
 * for bt_price_batch); sets the tuning of every depth from the smallest to
 * the largest N in it. */
int bt_autotune_batch(const bt_option *opts, int32_t n, int32_t precision, void *stream);
/* The tuning the library would use for depth N (after autotune or not). */
int bt_tuning_for(int32_t N, int32_t precision, bt_tuning *out);

/* ---- serving ------------------------------------------------------------
 * A continuous-batching request loop on one device.  A server thread admits
 * submitted requests while earlier ones are still on the GPU, as long as
 * device memory (mem_budget bytes of tables and scratch) and in-flight slots
 * allow; admitted requests are launched together as a batch on one of
 * `streams` HIP streams, so work of different batches overlaps on the device.
 * A batch holds either exact or MC requests (the class of the request that
 * has waited longest), so a short MC stage is never held back by a long
 * enumeration queued in its own batch.
 * Requests with N <= exact_max_n are priced exactly; deeper ones by
 * Partitioned MC: a pilot of 2^12 strata x 64 draws, then, if its relative
 * standard error exceeds mc_target_rel_se, a second estimate with 4 draws
 * per stratum and as many strata as the paths the pilot's error calls for
 * (at most mc_max_paths; a second estimate whose scratch would exceed
 * mem_budget is skipped and the pilot's estimate returned); the reported
 * std_err of an MC result is the square root of its var_unbiased.
 * Requests of a batch that fails to launch finish with the launch's error
 * code; those of a batch whose completion reports a HIP error, with
 * BT_EDEVICE.
 * Exact requests are priced with launch shapes made for one tree at a time
 * (bt_tuning {k, chunk}: {10, 128} for N = 11..25, {10, 256} for N = 26..27,
 * {10, 512} at N = 28 ({10, 256} in FP32), {11, 512} at N = 29, {16, 512}
 * for N = 30..31; the built-in shape otherwise), never with the built-in or
 * autotuned batch shapes, so each result is the same as bt_price_exact with
 * that tuning; an MC result is the same as the stratified estimate of its
 * stages priced alone. */
typedef struct {
    size_t mem_budget;        /* device bytes for in-flight requests       */
    int32_t max_inflight;     /* requests on the device at once            */
    int32_t streams;          /* 1..4                                      */
    int32_t precision;        /* bt_precision for every request            */
    int32_t exact_max_n;      /* <= 40; deeper requests go to MC           */
    double mc_target_rel_se;  /* e.g. 1e-4                                 */
    uint64_t mc_max_paths;    /* per-request cap on MC paths               */
    uint64_t mc_seed;         /* key of the MC draws; request id = stream  */
} bt_server_config;

typedef struct bt_server bt_server;

/* Timestamps (ns, CLOCK_MONOTONIC) of a finished request. */
typedef struct {
    int64_t t_submit, t_admit, t_done;
} bt_times;

int bt_server_create(const bt_server_config *cfg, bt_server **out);
/* Non-blocking; thread-safe.  *ticket identifies the request. */
int bt_server_submit(bt_server *srv, const bt_option *opt, uint64_t *ticket);
/* BT_OK with *out (and *times if non-NULL) filled once done, BT_EAGAIN
 * before, BT_ENOTFOUND for an unknown or already collected ticket. */
int bt_server_poll(bt_server *srv, uint64_t ticket, bt_result *out,
                   bt_times *times);
/* Counters: submitted, admitted, completed, peak device bytes in flight. */
int bt_server_stats(bt_server *srv, uint64_t *submitted, uint64_t *admitted,
                    uint64_t *completed, uint64_t *peak_bytes);
/* Stops the server thread after the in-flight work drains; pending
 * (unadmitted) requests complete with status BT_ESHUTDOWN. */
void bt_server_destroy(bt_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* BT_H */
