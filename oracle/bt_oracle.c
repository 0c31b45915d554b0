/*
 * bt_oracle.c -- plain, slow, serial reference for expected values over the
 * Bernoulli paths of a recombinant binomial tree.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: it exists so that tests, the smoke check and the CPU leg of
 * the benchmark have an independent answer to compare the GPU library with.
 * It shares no code, header, table or constant generator with the GPU path.
 *
 * What it computes, and where the paper defines it
 * ------------------------------------------------
 *  - tree parameters u, d = 1/u, p from (sigma, r, T, N): Section 2,
 *    assumptions A1-A3 and the u/p/beta display that follows them (Seydel's
 *    scheme), plus the Cox-Ross-Rubinstein choice u = exp(sigma sqrt(dt));
 *  - the price grid S_ij = S_0 u^j d^(i-j): Algorithm 1;
 *  - the path probability p^(x'1) (1-p)^(N - x'1): Section 2, the display
 *    before eq. (f11);
 *  - the value V(S_0) = e^{-qT} sum_x V_N(x) p(x): eq. (f13) (= eq. (expval)
 *    discounted);  the rank/prefix partition of Section 3 (eqs. (f14),(f15))
 *    is used only to split the sum over threads;
 *  - European values by backward induction on the Algorithm 1 grid and by the
 *    closed sum eq. (f8) (textbook pins, not the method);
 *  - lookback values by a lattice recursion over (level, running extreme)
 *    (textbook pin, not the method);
 *  - the Partitioned (stratified) Monte Carlo estimator, eqs. (mc9), (mc12)
 *    and its variance estimator, and basic MC, eq. (mc2), with
 *    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) as the generator;
 *  - proportional allocation R_m = R P(D_m) and the Shared-Sample estimator
 *    of the Remark in Section 4 (eq. (mc16));
 *  - the exact variance pieces that eqs. (mc13)-(mc15), (mc17)-(mc18) and
 *    Theorem 1 speak of;
 *  - eq. (f13) with time-varying up factors u_t and probabilities p_t (the
 *    case named after eq. (f12));
 *  - eq. (f13) over the 3^N paths of a trinomial tree (Section 3's remark
 *    on trees with more branches), with moment-matched parameters.
 *
 * Numbers: FP64 for every per-path quantity (the paper does not fix a
 * precision; FP64 is the reading), sums accumulated in x87 long double.
 */
#include "bt_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Section 2: tree parameters.                                         */
/* ------------------------------------------------------------------ */

/* Section 2, A1-A3: d = 1/u (A1), constant up-probability p (A2) chosen so
 * that E[S_{t+1} | S_t] = S_t e^{r dt} (A3), i.e. p = (e^{r dt} - d)/(u - d).
 * scheme 0: u = exp(sigma sqrt(dt)) (Cox, Ross, Rubinstein).
 * scheme 1: Seydel's u = beta + sqrt(beta^2 - 1) with
 *           beta = (e^{-r dt} + e^{(r + sigma^2) dt}) / 2.
 *           The paper prints "+1" under the root; with "+1", u d = 1 and the
 *           lognormal variance matching do not hold, and its printed exact
 *           values in Section 5 are reproduced only with "-1" (see tests). */
int orc_params(double sigma, double r, double T, int N, int scheme,
               double *u_out, double *p_out)
{
    if (!(sigma > 0) || !(T > 0) || N < 1 || !u_out || !p_out)
        return -1;
    double dt = T / (double)N;
    double u;
    if (scheme == ORC_SCHEME_CRR) {
        u = exp(sigma * sqrt(dt));
    } else if (scheme == ORC_SCHEME_SEYDEL) {
        double beta = 0.5 * (exp(-r * dt) + exp((r + sigma * sigma) * dt));
        u = beta + sqrt(beta * beta - 1.0);
    } else {
        return -1;
    }
    double d = 1.0 / u;
    double p = (exp(r * dt) - d) / (u - d);
    if (!(p > 0.0 && p < 1.0))
        return -2;
    *u_out = u;
    *p_out = p;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Section 2, Algorithm 1: the grid S_ij = S_0 u^j d^(i-j).            */
/* ------------------------------------------------------------------ */

typedef struct {
    int N;
    double *S;   /* S[i*(N+1) + j] for 0 <= j <= i <= N */
    double *w;   /* w[j] = p^j (1-p)^(N-j), j = 0..N: path probability */
} grid_t;

static int grid_build(const orc_option *o, grid_t *g)
{
    int N = o->N;
    g->N = N;
    g->S = (double *)malloc(sizeof(double) * (size_t)(N + 1) * (size_t)(N + 1));
    g->w = (double *)malloc(sizeof(double) * (size_t)(N + 1));
    if (!g->S || !g->w) {
        free(g->S);
        free(g->w);
        return -1;
    }
    double d = 1.0 / o->u;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= i; ++j)
            g->S[i * (N + 1) + j] = o->S * pow(o->u, j) * pow(d, i - j);
    for (int j = 0; j <= N; ++j)
        g->w[j] = pow(o->p, j) * pow(1.0 - o->p, N - j);
    return 0;
}

static void grid_free(grid_t *g)
{
    free(g->S);
    free(g->w);
}

static inline double grid_S(const grid_t *g, int i, int j)
{
    return g->S[i * (g->N + 1) + j];
}

/* ------------------------------------------------------------------ */
/* Payoffs.  Section 2, eqs. (call), (put); Section 5: the Asian put     */
/* (mean of S_1..S_N) and the fixed-strike lookback put (min of          */
/* S_1..S_N).  The Asian call and the floating lookback max_t S_t - S_N  */
/* use the same window t = 1..N.                                         */
/* ------------------------------------------------------------------ */

static double payoff_from_stats(int kind, double K, double sum, double mx,
                                double mn, double last, int N)
{
    double mean = sum / (double)N;
    switch (kind) {
    case ORC_ASIAN_CALL: return fmax(mean - K, 0.0);
    case ORC_ASIAN_PUT: return fmax(K - mean, 0.0);
    case ORC_LOOKBACK_FLOAT: return mx - last;
    case ORC_LOOKBACK_FIXED_PUT: return fmax(K - mn, 0.0);
    case ORC_EURO_CALL: return fmax(last - K, 0.0);
    case ORC_EURO_PUT: return fmax(K - last, 0.0);
    default: return NAN;
    }
}

/* x_t for t = 1..N from the path index x: the first step is the most
 * significant bit (Section 3: the rank bits z_{r-1}..z_0 are the leading
 * steps x_1..x_r, and the node index follows them). */
void orc_path_of_index(uint64_t x, int N, int *bits)
{
    for (int t = 1; t <= N; ++t)
        bits[t - 1] = (int)((x >> (N - t)) & 1u);
}

/* V_N(x) for one path, walking the grid step by step. */
static double payoff_of_bits(const orc_option *o, const grid_t *g,
                             const int *bits)
{
    int U = 0;
    double sum = 0.0, mx = -INFINITY, mn = INFINITY, last = o->S;
    for (int t = 1; t <= o->N; ++t) {
        U += bits[t - 1];
        double St = grid_S(g, t, U);
        sum += St;
        if (St > mx) mx = St;
        if (St < mn) mn = St;
        last = St;
    }
    return payoff_from_stats(o->payoff, o->K, sum, mx, mn, last, o->N);
}

static int count_ups(const int *bits, int N)
{
    int U = 0;
    for (int t = 0; t < N; ++t)
        U += bits[t];
    return U;
}

static int option_ok(const orc_option *o)
{
    return o && o->N >= 1 && o->N <= 64 && o->S > 0 && o->u > 1.0 &&
           o->p > 0.0 && o->p < 1.0 && o->T > 0 && o->payoff >= 0 &&
           o->payoff < ORC_NPAYOFF;
}

double orc_payoff_of_path(const orc_option *o, const int *bits)
{
    if (!option_ok(o)) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    double v = payoff_of_bits(o, &g, bits);
    grid_free(&g);
    return v;
}

double orc_prob_of_path(const orc_option *o, const int *bits)
{
    if (!option_ok(o)) return NAN;
    int U = count_ups(bits, o->N);
    return pow(o->p, U) * pow(1.0 - o->p, o->N - U);
}

/* ------------------------------------------------------------------ */
/* Eq. (f13), naive form: one path at a time, O(N) per path, as in the  */
/* paper's own loop (build the path from its index, take its           */
/* probability and its payoff, accumulate).  Compensated long double   */
/* sum (Neumaier) so that the reference is far tighter than 1e-12.      */
/* ------------------------------------------------------------------ */

typedef struct {
    long double s, c;
} ksum_t;

static inline void ksum_add(ksum_t *k, long double v)
{
    long double t = k->s + v;
    if (fabsl(k->s) >= fabsl(v))
        k->c += (k->s - t) + v;
    else
        k->c += (v - t) + k->s;
    k->s = t;
}

static inline long double ksum_get(const ksum_t *k) { return k->s + k->c; }

/* Undiscounted sum over x in [x_begin, x_end) of p(x) V_N(x). */
static long double naive_range(const orc_option *o, const grid_t *g,
                               uint64_t x_begin, uint64_t x_end)
{
    int bits[64];
    ksum_t acc = {0.0L, 0.0L};
    for (uint64_t x = x_begin; x < x_end; ++x) {
        orc_path_of_index(x, o->N, bits);
        double px = g->w[count_ups(bits, o->N)];
        double v = payoff_of_bits(o, g, bits);
        ksum_add(&acc, (long double)px * (long double)v);
    }
    return ksum_get(&acc);
}

double orc_price_naive(const orc_option *o)
{
    if (!option_ok(o) || o->N > 40) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    long double s = naive_range(o, &g, 0, (uint64_t)1 << o->N);
    grid_free(&g);
    return (double)((long double)exp(-o->r * o->T) * s);
}

double orc_range_naive(const orc_option *o, uint64_t x_begin, uint64_t x_end)
{
    if (!option_ok(o) || o->N > 40) return NAN;
    uint64_t n = (uint64_t)1 << o->N;
    if (x_end > n || x_begin > x_end) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    long double s = naive_range(o, &g, x_begin, x_end);
    grid_free(&g);
    return (double)s;
}

/* ------------------------------------------------------------------ */
/* Eq. (f13), depth-first form: the same sum, visiting the leaves in    */
/* index order while carrying the running sum / max / min of S_t down   */
/* the tree (amortised O(1) per leaf).  Each node returns the sum of    */
/* its two subtrees, so the summation is pairwise by construction.     */
/* ------------------------------------------------------------------ */

typedef struct {
    const orc_option *o;
    const grid_t *g;
} dfs_ctx;

static long double dfs_node(const dfs_ctx *c, int t, int U, double sum,
                            double mx, double mn, double last)
{
    const orc_option *o = c->o;
    if (t == o->N)
        return (long double)c->g->w[U] *
               (long double)payoff_from_stats(o->payoff, o->K, sum, mx, mn,
                                              last, o->N);
    long double acc = 0.0L;
    for (int b = 0; b <= 1; ++b) { /* b = 0: down first (lower index) */
        int U1 = U + b;
        double St = grid_S(c->g, t + 1, U1);
        acc += dfs_node(c, t + 1, U1, sum + St, St > mx ? St : mx,
                        St < mn ? St : mn, St);
    }
    return acc;
}

/* Walk the first `depth` steps of prefix z and return the node state. */
static void walk_prefix(const grid_t *g, double S0, uint64_t z,
                        int depth, int *U, double *sum, double *mx, double *mn,
                        double *last)
{
    *U = 0;
    *sum = 0.0;
    *mx = -INFINITY;
    *mn = INFINITY;
    *last = S0;
    for (int t = 1; t <= depth; ++t) {
        *U += (int)((z >> (depth - t)) & 1u);
        double St = grid_S(g, t, *U);
        *sum += St;
        if (St > *mx) *mx = St;
        if (St < *mn) *mn = St;
        *last = St;
    }
}

static long double dfs_subtree(const orc_option *o, const grid_t *g, int depth,
                               uint64_t z)
{
    dfs_ctx c = {o, g};
    int U;
    double sum, mx, mn, last;
    walk_prefix(g, o->S, z, depth, &U, &sum, &mx, &mn, &last);
    return dfs_node(&c, depth, U, sum, mx, mn, last);
}

/* Section 3 with threads as ranks: rank m owns the 2^(N-r) paths whose
 * first r steps spell m (MSB first); each rank sums its block (eq. (f14)),
 * and the block sums are combined pairwise in rank order (eq. (f15)), so the
 * result does not depend on how many threads ran. */
typedef struct {
    const orc_option *o;
    const grid_t *g;
    int depth;
    uint64_t first, count; /* prefixes handled by this thread */
    long double *out;      /* out[z] for z in [first, first+count) */
} rank_job;

static void *rank_worker(void *arg)
{
    rank_job *j = (rank_job *)arg;
    for (uint64_t z = j->first; z < j->first + j->count; ++z)
        j->out[z] = dfs_subtree(j->o, j->g, j->depth, z);
    return NULL;
}

static long double pairwise(const long double *v, uint64_t n)
{
    if (n == 1) return v[0];
    uint64_t h = n / 2;
    return pairwise(v, h) + pairwise(v + h, n - h);
}

static long double dfs_sum(const orc_option *o, const grid_t *g, int threads)
{
    int N = o->N;
    int depth = N < 10 ? N : 10; /* 2^depth prefix blocks (ranks) */
    uint64_t M = (uint64_t)1 << depth;
    long double *part = (long double *)malloc(sizeof(long double) * M);
    if (!part) return NAN;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > M) threads = (int)M;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    rank_job *jobs = (rank_job *)malloc(sizeof(rank_job) * (size_t)threads);
    uint64_t per = M / (uint64_t)threads, extra = M % (uint64_t)threads;
    uint64_t first = 0;
    for (int t = 0; t < threads; ++t) {
        uint64_t cnt = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (rank_job){o, g, depth, first, cnt, part};
        first += cnt;
        if (threads > 1)
            pthread_create(&tid[t], NULL, rank_worker, &jobs[t]);
        else
            rank_worker(&jobs[t]);
    }
    if (threads > 1)
        for (int t = 0; t < threads; ++t)
            pthread_join(tid[t], NULL);
    long double s = pairwise(part, M);
    free(part);
    free(tid);
    free(jobs);
    return s;
}

double orc_price_dfs(const orc_option *o, int threads)
{
    if (!option_ok(o) || o->N > 40) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    long double s = dfs_sum(o, &g, threads);
    grid_free(&g);
    return (double)((long double)exp(-o->r * o->T) * s);
}

/* Undiscounted sum of p(x) V_N(x) over the 2^(N-depth) paths whose first
 * `depth` steps spell z (eq. (f14) without the discount). */
double orc_subtree_sum(const orc_option *o, int depth, uint64_t z)
{
    if (!option_ok(o) || depth < 0 || depth > o->N || o->N > 40) return NAN;
    if (depth < 64 && z >= ((uint64_t)1 << depth)) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    long double s = dfs_subtree(o, &g, depth, z);
    grid_free(&g);
    return (double)s;
}

/* ------------------------------------------------------------------ */
/* European pins: eq. (f8) closed sum and backward induction.          */
/* ------------------------------------------------------------------ */

static double leaf_payoff(int kind, double K, double SN)
{
    if (kind == ORC_EURO_CALL) return fmax(SN - K, 0.0);
    if (kind == ORC_EURO_PUT) return fmax(K - SN, 0.0);
    return NAN;
}

/* Eq. (f8): e^{-qT} sum_i C(N,i) p^i (1-p)^{N-i} V_{Ni}. */
double orc_euro_closed(const orc_option *o)
{
    if (!option_ok(o)) return NAN;
    if (o->payoff != ORC_EURO_CALL && o->payoff != ORC_EURO_PUT) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    long double acc = 0.0L, binom = 1.0L; /* C(N, i) */
    for (int i = 0; i <= o->N; ++i) {
        acc += binom * (long double)g.w[i] *
               (long double)leaf_payoff(o->payoff, o->K, grid_S(&g, o->N, i));
        binom = binom * (long double)(o->N - i) / (long double)(i + 1);
    }
    grid_free(&g);
    return (double)((long double)exp(-o->r * o->T) * acc);
}

/* Backward induction on the Algorithm 1 grid: V_{N,j} = payoff(S_{N,j}),
 * V_{i,j} = e^{-r dt} (p V_{i+1,j+1} + (1-p) V_{i+1,j}). */
double orc_euro_backward(const orc_option *o)
{
    if (!option_ok(o)) return NAN;
    if (o->payoff != ORC_EURO_CALL && o->payoff != ORC_EURO_PUT) return NAN;
    grid_t g;
    if (grid_build(o, &g)) return NAN;
    int N = o->N;
    double *V = (double *)malloc(sizeof(double) * (size_t)(N + 1));
    for (int j = 0; j <= N; ++j)
        V[j] = leaf_payoff(o->payoff, o->K, grid_S(&g, N, j));
    double disc1 = exp(-o->r * o->T / (double)N);
    for (int i = N - 1; i >= 0; --i)
        for (int j = 0; j <= i; ++j)
            V[j] = disc1 * (o->p * V[j + 1] + (1.0 - o->p) * V[j]);
    double v = V[0];
    free(V);
    grid_free(&g);
    return v;
}

/* ------------------------------------------------------------------ */
/* Lookback pin: forward recursion over (level, running extreme level). */
/* A textbook lattice method, independent of path enumeration.  The     */
/* extreme is taken over t = 1..N (S_0 excluded), as for enumeration.    */
/* Returns the discounted first moment; second moment (undiscounted      */
/* E[V^2]) in *m2 if non-NULL.                                           */
/* ------------------------------------------------------------------ */

double orc_lookback_dp(const orc_option *o, double *m2)
{
    if (!option_ok(o)) return NAN;
    if (o->payoff != ORC_LOOKBACK_FLOAT && o->payoff != ORC_LOOKBACK_FIXED_PUT)
        return NAN;
    int N = o->N, W = 2 * N + 1; /* levels -N..N stored at +N */
    int want_max = (o->payoff == ORC_LOOKBACK_FLOAT);
    size_t cells = (size_t)W * (size_t)W;
    long double *cur = (long double *)calloc(cells, sizeof(long double));
    long double *nxt = (long double *)calloc(cells, sizeof(long double));
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return NAN;
    }
    /* t = 1: level +-1, extreme = that level. */
    cur[(size_t)(N + 1) * W + (N + 1)] = o->p;
    cur[(size_t)(N - 1) * W + (N - 1)] = 1.0 - o->p;
    for (int t = 1; t < N; ++t) {
        memset(nxt, 0, cells * sizeof(long double));
        for (int l = -t; l <= t; ++l)
            for (int e = -t; e <= t; ++e) {
                long double m = cur[(size_t)(l + N) * W + (e + N)];
                if (m == 0.0L) continue;
                for (int b = 0; b <= 1; ++b) {
                    int l1 = l + (b ? 1 : -1);
                    int e1 = want_max ? (l1 > e ? l1 : e) : (l1 < e ? l1 : e);
                    nxt[(size_t)(l1 + N) * W + (e1 + N)] +=
                        m * (long double)(b ? o->p : 1.0 - o->p);
                }
            }
        long double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    long double s1 = 0.0L, s2 = 0.0L;
    for (int l = -N; l <= N; ++l)
        for (int e = -N; e <= N; ++e) {
            long double m = cur[(size_t)(l + N) * W + (e + N)];
            if (m == 0.0L) continue;
            double Se = o->S * pow(o->u, e), Sl = o->S * pow(o->u, l);
            double v = want_max ? Se - Sl : fmax(o->K - Se, 0.0);
            s1 += m * (long double)v;
            s2 += m * (long double)v * (long double)v;
        }
    free(cur);
    free(nxt);
    if (m2) *m2 = (double)s2;
    return (double)((long double)exp(-o->r * o->T) * s1);
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from its definition (Salmon et al., SC'11): ten        */
/* rounds of two 32x32->64 multiplies and a Feistel-like swap, the key   */
/* advanced by the Weyl constants between rounds.                        */
/* ------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Up-move threshold: a step goes up iff its 32-bit uniform word is below
 * floor(p 2^32), so P(up) = floor(p 2^32) / 2^32. */
uint32_t orc_up_threshold(double p)
{
    double t = floor(ldexp(p, 32));
    if (t >= 4294967296.0) return 0xFFFFFFFFu;
    if (t < 0) return 0;
    return (uint32_t)t;
}

/* Bits of the suffix of sample m in stratum z.  Step j (0-based, j < L)
 * reads the 16-bit half h_j of word (j % 8) / 2 of the Philox block with
 * counter (j / 8, m, z, stream) and key (seed low 32 bits, seed high 32
 * bits): the high half for even j, the low half for odd j.  With
 * thr = floor(p 2^32) split into halves thr_hi, thr_lo, the step goes up iff
 * h_j < thr_hi; on a tie (h_j == thr_hi) it goes up iff g_j < thr_lo, where
 * g_j is the high half of word 0 of the block with counter
 * (2^31 + j, m, z, stream).  The step's uniform is the 32-bit number
 * (h_j, g_j), so P(up) = thr / 2^32 exactly; g_j is drawn only when it
 * decides (probability 2^-16). */
void orc_mc_suffix_bits(uint64_t seed, uint32_t stream, uint32_t z, uint32_t m,
                        int L, uint32_t thr, int *bits)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t blk[4];
    const uint32_t thr_hi = thr >> 16, thr_lo = thr & 0xFFFFu;
    for (int j = 0; j < L; ++j) {
        if (j % 8 == 0) {
            uint32_t ctr[4] = {(uint32_t)(j / 8), m, z, stream};
            orc_philox4x32_10(ctr, key, blk);
        }
        const uint32_t w = blk[(j % 8) / 2];
        const uint32_t h = (j % 2 == 0) ? (w >> 16) : (w & 0xFFFFu);
        if (h != thr_hi) {
            bits[j] = h < thr_hi ? 1 : 0;
        } else {
            uint32_t ctr[4] = {0x80000000u + (uint32_t)j, m, z, stream}, g[4];
            orc_philox4x32_10(ctr, key, g);
            bits[j] = (g[0] >> 16) < thr_lo ? 1 : 0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Section 4: Partitioned Monte Carlo with R_m draws in every stratum.  */
/*   theta_s = sum_z P(D_z) thetahat_z                      eq. (mc12)  */
/*   Var(theta_s) = sum_z P(D_z)^2 Var[V | D_z] / R_m   (first line of  */
/*                  eq. (mc13), before proportional allocation)         */
/* estimated with the plug-in s_z^2 = (1/R_m) sum (V - thetahat_z)^2    */
/* (the paper's normalisation) and with 1/(R_m - 1) beside it.  r = 0 is */
/* basic MC, eq. (mc2) and the estimator printed after it.             */
/* ------------------------------------------------------------------ */

int orc_mc_stratified_range(const orc_option *o, int r, uint32_t Rm,
                            uint64_t seed, uint32_t stream, uint64_t z_begin,
                            uint64_t z_end, orc_mc_sums *out)
{
    if (!option_ok(o) || r < 0 || r >= o->N || r > 32 || Rm < 1 || !out)
        return -1;
    uint64_t nz = (uint64_t)1 << r;
    if (z_end > nz || z_begin > z_end) return -1;
    grid_t g;
    if (grid_build(o, &g)) return -1;
    int N = o->N, L = N - r;
    uint32_t thr = orc_up_threshold(o->p);
    int bits[64];
    double *v = (double *)malloc(sizeof(double) * Rm);
    ksum_t est = {0, 0}, var_pi = {0, 0}, var_ub = {0, 0}, sec = {0, 0};
    for (uint64_t z = z_begin; z < z_end; ++z) {
        orc_path_of_index(z, r, bits);
        int a = count_ups(bits, r);
        double Wz = pow(o->p, a) * pow(1.0 - o->p, r - a); /* P(D_z) */
        for (uint32_t m = 0; m < Rm; ++m) {
            orc_mc_suffix_bits(seed, stream, (uint32_t)z, m, L, thr, bits + r);
            v[m] = payoff_of_bits(o, &g, bits);
        }
        long double mean = 0.0L;
        for (uint32_t m = 0; m < Rm; ++m) mean += v[m];
        mean /= (long double)Rm;
        long double ss = 0.0L;
        for (uint32_t m = 0; m < Rm; ++m) {
            long double dv = (long double)v[m] - mean;
            ss += dv * dv;
        }
        long double sq = 0.0L;
        for (uint32_t m = 0; m < Rm; ++m) sq += (long double)v[m] * (long double)v[m];
        ksum_add(&est, (long double)Wz * mean);
        long double W2 = (long double)Wz * (long double)Wz;
        ksum_add(&var_pi, W2 * (ss / (long double)Rm) / (long double)Rm);
        if (Rm > 1)
            ksum_add(&var_ub, W2 * (ss / (long double)(Rm - 1)) / (long double)Rm);
        ksum_add(&sec, (long double)Wz * (sq / (long double)Rm));
    }
    free(v);
    grid_free(&g);
    out->theta = (double)ksum_get(&est);
    out->var_plugin = (double)ksum_get(&var_pi);
    out->var_unbiased = Rm > 1 ? (double)ksum_get(&var_ub) : NAN;
    out->second = (double)ksum_get(&sec);
    return 0;
}

int orc_mc_stratified(const orc_option *o, int r, uint32_t Rm, uint64_t seed,
                      uint32_t stream, orc_mc_result *res)
{
    if (!res || !option_ok(o) || r < 0 || r >= o->N || r > 32) return -1;
    orc_mc_sums s;
    int rc = orc_mc_stratified_range(o, r, Rm, seed, stream, 0,
                                     (uint64_t)1 << r, &s);
    if (rc) return rc;
    double disc = exp(-o->r * o->T);
    res->value = disc * s.theta;
    res->var_plugin = disc * disc * s.var_plugin;
    res->var_unbiased = disc * disc * s.var_unbiased;
    /* plain MC over the same number of paths: Var[V] estimated from the
     * strata as E[V^2] - E[V]^2, divided by the paths */
    long double vv = (long double)s.second - (long double)s.theta * (long double)s.theta;
    res->var_plain = disc * disc * (double)(vv / ((long double)Rm * ldexpl(1.0L, r)));
    return 0;
}

/* ------------------------------------------------------------------ */
/* Section 4, proportional allocation R_m = R P(D_m) (the allocation the */
/* text chooses before eq. (mc13)).  R P(D_m) is rounded to the nearest  */
/* integer and raised to at least 1, so that every stratum is sampled   */
/* (reading: the paper ignores the rounding).  Returns the estimate, the */
/* general plug-in variance sum_m P(D_m)^2 s_m^2 / R_m, its 1/(R_m - 1)  */
/* form, and the paper's shortcut (1/R^2) sum_m sum_i (V - thetahat_m)^2 */
/* (exact only under exact proportionality).  Undiscounted.              */
/* ------------------------------------------------------------------ */

static uint32_t proportional_rm(double R, double W)
{
    double x = floor(R * W + 0.5);
    if (x < 1.0) x = 1.0;
    if (x > 4294967295.0) x = 4294967295.0;
    return (uint32_t)x;
}

/* Strata [z_begin, z_end) only (their sums; the whole estimator is the   */
/* range over all 2^r strata).                                           */
int orc_mc_proportional_range(const orc_option *o, int r, uint64_t R, uint64_t seed,
                              uint32_t stream, uint64_t z_begin, uint64_t z_end,
                              orc_mc_prop *out)
{
    if (!option_ok(o) || r < 0 || r >= o->N || r > 30 || R < 1 || !out) return -1;
    uint64_t nz = (uint64_t)1 << r, used = 0;
    if (z_end > nz || z_begin > z_end) return -1;
    grid_t g;
    if (grid_build(o, &g)) return -1;
    int N = o->N, L = N - r;
    uint32_t thr = orc_up_threshold(o->p);
    int bits[64];
    uint32_t rmax = 0;
    ksum_t est = {0, 0}, vpi = {0, 0}, vub = {0, 0}, vpaper = {0, 0}, sec = {0, 0};
    for (uint64_t z = z_begin; z < z_end; ++z) {
        orc_path_of_index(z, r, bits);
        int a = count_ups(bits, r);
        double Wz = pow(o->p, a) * pow(1.0 - o->p, r - a);
        uint32_t Rm = proportional_rm((double)R, Wz);
        long double sum = 0.0L, sq = 0.0L;
        double *v = (double *)malloc(sizeof(double) * Rm);
        for (uint32_t m = 0; m < Rm; ++m) {
            orc_mc_suffix_bits(seed, stream, (uint32_t)z, m, L, thr, bits + r);
            v[m] = payoff_of_bits(o, &g, bits);
            sum += v[m];
            sq += (long double)v[m] * (long double)v[m];
        }
        long double mean = sum / (long double)Rm, ss = 0.0L;
        for (uint32_t m = 0; m < Rm; ++m) {
            long double dv = (long double)v[m] - mean;
            ss += dv * dv;
        }
        free(v);
        long double W2 = (long double)Wz * (long double)Wz;
        ksum_add(&est, (long double)Wz * mean);
        ksum_add(&vpi, W2 * (ss / (long double)Rm) / (long double)Rm);
        if (Rm > 1) ksum_add(&vub, W2 * (ss / (long double)(Rm - 1)) / (long double)Rm);
        ksum_add(&vpaper, ss / ((long double)R * (long double)R));
        ksum_add(&sec, (long double)Wz * (sq / (long double)Rm));
        used += Rm;
        if (Rm > rmax) rmax = Rm;
    }
    grid_free(&g);
    out->theta = (double)ksum_get(&est);
    out->var_plugin = (double)ksum_get(&vpi);
    /* strata with one draw add nothing to the 1/(R_m - 1) form; with no
     * stratum above one draw it is undefined, as for equal allocation */
    out->var_unbiased = rmax > 1 ? (double)ksum_get(&vub) : NAN;
    out->var_paper = (double)ksum_get(&vpaper);
    out->second = (double)ksum_get(&sec);
    out->samples = used;
    return 0;
}

int orc_mc_proportional(const orc_option *o, int r, uint64_t R, uint64_t seed,
                        uint32_t stream, orc_mc_prop *out)
{
    if (r < 0 || r > 30) return -1;
    return orc_mc_proportional_range(o, r, R, seed, stream, 0, (uint64_t)1 << r, out);
}

/* ------------------------------------------------------------------ */
/* Shared-Sample MC (Section 4, Remark, eq. (mc16)): one set of R suffix */
/* draws y_i, each combined with every prefix z:                         */
/*   h_i = sum_z P(D_z) V(z, y_i),  thetatilde = (1/R) sum_i h_i,        */
/*   Var-hat = (1/R^2) sum_i (h_i - thetatilde)^2                        */
/* (reading: the estimator printed after eq. (mc16) subtracts the        */
/* overall estimate).  Draw i is the suffix of orc_mc_suffix_bits with  */
/* m = i and z = 0xFFFFFFFF.  Undiscounted.                              */
/* ------------------------------------------------------------------ */

/* h_i = sum_z P(D_z) V(z, y_i) for the shared draws i in [i_begin,      */
/* i_end), into h[i - i_begin] (undiscounted).                           */
static void shared_h(const orc_option *o, const grid_t *g, int r, uint64_t seed,
                     uint32_t stream, uint32_t i_begin, uint32_t i_end, long double *h)
{
    int N = o->N, L = N - r;
    uint32_t thr = orc_up_threshold(o->p);
    uint64_t nz = (uint64_t)1 << r;
    int bits[64];
    for (uint32_t i = i_begin; i < i_end; ++i) {
        orc_mc_suffix_bits(seed, stream, 0xFFFFFFFFu, i, L, thr, bits + r);
        ksum_t hi = {0, 0};
        for (uint64_t z = 0; z < nz; ++z) {
            orc_path_of_index(z, r, bits);
            int a = count_ups(bits, r);
            double Wz = pow(o->p, a) * pow(1.0 - o->p, r - a);
            ksum_add(&hi, (long double)Wz * (long double)payoff_of_bits(o, g, bits));
        }
        h[i - i_begin] = ksum_get(&hi);
    }
}

int orc_mc_shared_draws(const orc_option *o, int r, uint64_t seed, uint32_t stream,
                        uint32_t i_begin, uint32_t i_end, double *h_out)
{
    if (!option_ok(o) || r < 0 || r >= o->N || r > 24 || i_begin > i_end || !h_out) return -1;
    grid_t g;
    if (grid_build(o, &g)) return -1;
    long double *h = (long double *)malloc(sizeof(long double) * (i_end - i_begin + 1));
    shared_h(o, &g, r, seed, stream, i_begin, i_end, h);
    for (uint32_t i = i_begin; i < i_end; ++i) h_out[i - i_begin] = (double)h[i - i_begin];
    free(h);
    grid_free(&g);
    return 0;
}

int orc_mc_shared(const orc_option *o, int r, uint32_t R, uint64_t seed, uint32_t stream,
                  orc_mc_sums *out)
{
    if (!option_ok(o) || r < 0 || r >= o->N || r > 24 || R < 1 || !out) return -1;
    grid_t g;
    if (grid_build(o, &g)) return -1;
    long double *h = (long double *)malloc(sizeof(long double) * R);
    shared_h(o, &g, r, seed, stream, 0, R, h);
    long double tot = 0.0L;
    for (uint32_t i = 0; i < R; ++i) tot += h[i];
    long double mean = tot / (long double)R, ss = 0.0L;
    for (uint32_t i = 0; i < R; ++i) ss += (h[i] - mean) * (h[i] - mean);
    free(h);
    grid_free(&g);
    out->theta = (double)mean;
    out->var_plugin = (double)(ss / ((long double)R * (long double)R));
    out->var_unbiased = R > 1 ? (double)(ss / ((long double)R * (long double)(R - 1))) : NAN;
    out->second = NAN; /* no per-stratum draws to estimate E[V^2] from */
    return 0;
}

/* ------------------------------------------------------------------ */
/* Exact variance pieces for a stratification of depth r, by complete   */
/* enumeration: the exact counterparts of what the MC estimators         */
/* estimate (eqs. (mc2), (mc13)-(mc15)).  All undiscounted.              */
/*   var_total   = Var[V(X)]                                            */
/*   within      = sum_z P(D_z) Var[V | D_z]                            */
/*   between     = Var_D E[V | D]                                       */
/*   within_sq   = sum_z P(D_z)^2 Var[V | D_z]                          */
/* ------------------------------------------------------------------ */

int orc_exact_strata(const orc_option *o, int r, orc_strata_exact *out)
{
    if (!option_ok(o) || r < 0 || r > o->N || o->N > 30 || !out) return -1;
    grid_t g;
    if (grid_build(o, &g)) return -1;
    int N = o->N, L = N - r;
    uint64_t nz = (uint64_t)1 << r, ns = (uint64_t)1 << L;
    int bits[64];
    /* h(s) = sum_z P(z) V(z, s) and the within-suffix second moment, by suffix */
    long double *h = (long double *)calloc(ns, sizeof(long double));
    long double *h2 = (long double *)calloc(ns, sizeof(long double));
    long double E1 = 0, E2 = 0, within = 0, within_sq = 0, between_m2 = 0;
    for (uint64_t z = 0; z < nz; ++z) {
        orc_path_of_index(z, r, bits);
        int a = count_ups(bits, r);
        long double Wz = (long double)pow(o->p, a) * (long double)pow(1.0 - o->p, r - a);
        long double m1 = 0, m2 = 0; /* conditional moments given D_z */
        for (uint64_t s = 0; s < ns; ++s) {
            orc_path_of_index(s, L, bits + r);
            int b = count_ups(bits + r, L);
            long double ws = (long double)pow(o->p, b) * (long double)pow(1.0 - o->p, L - b);
            long double v = payoff_of_bits(o, &g, bits);
            m1 += ws * v;
            m2 += ws * v * v;
            h[s] += Wz * v;
            h2[s] += Wz * v * v;
        }
        long double vz = m2 - m1 * m1;
        E1 += Wz * m1;
        E2 += Wz * m2;
        within += Wz * vz;
        within_sq += Wz * Wz * vz;
        between_m2 += Wz * m1 * m1;
    }
    long double sh1 = 0, sh2 = 0, wy = 0;
    for (uint64_t s = 0; s < ns; ++s) {
        orc_path_of_index(s, L, bits + r);
        int b = count_ups(bits + r, L);
        long double ws = (long double)pow(o->p, b) * (long double)pow(1.0 - o->p, L - b);
        sh1 += ws * h[s];
        sh2 += ws * h[s] * h[s];
        wy += ws * (h2[s] - h[s] * h[s]);
    }
    free(h);
    free(h2);
    grid_free(&g);
    out->mean = (double)E1;
    out->var_total = (double)(E2 - E1 * E1);
    out->within = (double)within;
    out->between = (double)(between_m2 - E1 * E1);
    out->within_sq = (double)within_sq;
    out->shared = (double)(sh2 - sh1 * sh1);
    out->within_y = (double)wy;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. (f13) with time-varying moves (the case the text after eq. (f12) */
/* names): step t = 1..N multiplies the price by u_t (up, probability   */
/* p_t) or by d_t = 1/u_t (down), and                                   */
/*   p(x) = prod_t p_t^{I(x_t = 1)} (1 - p_t)^{I(x_t = 0)}.             */
/* The tree need not recombine; the path sum does not need it to.       */
/* Prices by repeated multiplication along the path, weights as running */
/* products.  Two forms: one path at a time (naive), and depth-first    */
/* with threads as ranks over the first min(N, 10) steps (as above).    */
/* ------------------------------------------------------------------ */

static int tv_ok(const orc_option *o, const double *u, const double *p)
{
    if (!o || !u || !p || o->N < 1 || o->N > 40 || !(o->S > 0) || !(o->T > 0) ||
        o->payoff < 0 || o->payoff >= ORC_NPAYOFF)
        return 0;
    for (int t = 0; t < o->N; ++t)
        if (!(u[t] > 1.0) || !(p[t] > 0.0 && p[t] < 1.0) || !isfinite(u[t])) return 0;
    return 1;
}

static long double tv_path(const orc_option *o, const double *u, const double *p,
                           const int *bits)
{
    double S = o->S, w = 1.0, sum = 0.0, mx = -INFINITY, mn = INFINITY;
    for (int t = 0; t < o->N; ++t) {
        if (bits[t]) {
            S = S * u[t];
            w = w * p[t];
        } else {
            S = S / u[t];
            w = w * (1.0 - p[t]);
        }
        sum += S;
        if (S > mx) mx = S;
        if (S < mn) mn = S;
    }
    return (long double)w *
           (long double)payoff_from_stats(o->payoff, o->K, sum, mx, mn, S, o->N);
}

double orc_price_tv_naive(const orc_option *o, const double *u, const double *p)
{
    if (!tv_ok(o, u, p) || o->N > 30) return NAN;
    int bits[64];
    ksum_t acc = {0.0L, 0.0L};
    for (uint64_t x = 0; x < ((uint64_t)1 << o->N); ++x) {
        orc_path_of_index(x, o->N, bits);
        ksum_add(&acc, tv_path(o, u, p, bits));
    }
    return (double)((long double)exp(-o->r * o->T) * ksum_get(&acc));
}

typedef struct {
    const orc_option *o;
    const double *u, *p;
} tv_ctx;

/* Sum over the subtree below a node at step t (t steps taken). */
static long double tv_node(const tv_ctx *c, int t, double S, double w, double sum,
                           double mx, double mn)
{
    const orc_option *o = c->o;
    if (t == o->N)
        return (long double)w *
               (long double)payoff_from_stats(o->payoff, o->K, sum, mx, mn, S, o->N);
    long double acc = 0.0L;
    for (int b = 0; b <= 1; ++b) { /* down first: lower index */
        double St = b ? S * c->u[t] : S / c->u[t];
        double wt = b ? w * c->p[t] : w * (1.0 - c->p[t]);
        acc += tv_node(c, t + 1, St, wt, sum + St, St > mx ? St : mx, St < mn ? St : mn);
    }
    return acc;
}

typedef struct {
    const tv_ctx *c;
    int depth;
    uint64_t first, count;
    long double *out;
} tv_job;

static void *tv_worker(void *arg)
{
    tv_job *j = (tv_job *)arg;
    const tv_ctx *c = j->c;
    for (uint64_t z = j->first; z < j->first + j->count; ++z) {
        double S = c->o->S, w = 1.0, sum = 0.0, mx = -INFINITY, mn = INFINITY;
        for (int t = 0; t < j->depth; ++t) {
            int b = (int)((z >> (j->depth - 1 - t)) & 1u);
            S = b ? S * c->u[t] : S / c->u[t];
            w = b ? w * c->p[t] : w * (1.0 - c->p[t]);
            sum += S;
            if (S > mx) mx = S;
            if (S < mn) mn = S;
        }
        j->out[z] = tv_node(c, j->depth, S, w, sum, mx, mn);
    }
    return NULL;
}

double orc_price_tv(const orc_option *o, const double *u, const double *p, int threads)
{
    if (!tv_ok(o, u, p)) return NAN;
    tv_ctx c = {o, u, p};
    int depth = o->N < 10 ? o->N : 10;
    uint64_t M = (uint64_t)1 << depth;
    long double *part = (long double *)malloc(sizeof(long double) * M);
    if (!part) return NAN;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > M) threads = (int)M;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    tv_job *jobs = (tv_job *)malloc(sizeof(tv_job) * (size_t)threads);
    uint64_t per = M / (uint64_t)threads, extra = M % (uint64_t)threads, first = 0;
    for (int t = 0; t < threads; ++t) {
        uint64_t cnt = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (tv_job){&c, depth, first, cnt, part};
        first += cnt;
        if (threads > 1)
            pthread_create(&tid[t], NULL, tv_worker, &jobs[t]);
        else
            tv_worker(&jobs[t]);
    }
    if (threads > 1)
        for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
    long double s = pairwise(part, M);
    free(part);
    free(tid);
    free(jobs);
    return (double)((long double)exp(-o->r * o->T) * s);
}

/* ------------------------------------------------------------------ */
/* Trinomial trees (Section 3 notes that the path partition applies to  */
/* trees with more than two branches, citing Boyle's trinomial tree).   */
/* Each step moves the price by u (up, probability pu), 1 (middle,      */
/* pm = 1 - pu - pd) or 1/u (down, pd).  A path is N base-3 digits,     */
/* first step most significant, digit 0 = down, 1 = middle, 2 = up; its */
/* probability is the product of the step probabilities and eq. (f13)   */
/* sums over all 3^N paths.                                            */
/* ------------------------------------------------------------------ */

/* u = exp(lambda sigma sqrt(dt)) and (pu, pd) matching the mean e^{r dt}
 * and the second moment e^{(2r + sigma^2) dt} of the lognormal step
 * (Boyle's stretch parameter lambda), by solving the 2x2 linear system
 *   pu (u - 1)   + pd (1/u - 1)   = M - 1
 *   pu (u^2 - 1) + pd (1/u^2 - 1) = M^2 e^{sigma^2 dt} - 1.            */
int orc_params_trinomial(double sigma, double r, double T, int N, double lambda,
                         double *u_out, double *pu_out, double *pd_out)
{
    if (!(sigma > 0) || !(T > 0) || N < 1 || !(lambda > 0) || !u_out || !pu_out || !pd_out)
        return -1;
    double dt = T / (double)N;
    double u = exp(lambda * sigma * sqrt(dt));
    double M = exp(r * dt), V2 = M * M * exp(sigma * sigma * dt);
    double a11 = u - 1.0, a12 = 1.0 / u - 1.0, b1 = M - 1.0;
    double a21 = u * u - 1.0, a22 = 1.0 / (u * u) - 1.0, b2 = V2 - 1.0;
    double det = a11 * a22 - a12 * a21;
    double pu = (b1 * a22 - a12 * b2) / det;
    double pd = (a11 * b2 - b1 * a21) / det;
    if (!(pu > 0.0) || !(pd > 0.0) || !(pu + pd < 1.0)) return -2;
    *u_out = u;
    *pu_out = pu;
    *pd_out = pd;
    return 0;
}

static int tri_ok(const orc_option *o, double pd)
{
    /* o->p is pu; the middle probability may be zero (binomial limit) */
    return o && o->N >= 1 && o->N <= 30 && o->S > 0 && o->u > 1.0 && o->T > 0 &&
           o->p > 0.0 && pd > 0.0 && o->p + pd <= 1.0 && o->payoff >= 0 &&
           o->payoff < ORC_NPAYOFF;
}

/* digits[t] for t = 0..N-1 (step t+1) of path index x in base 3 */
void orc_tri_digits(uint64_t x, int N, int *digits)
{
    for (int t = N - 1; t >= 0; --t) {
        digits[t] = (int)(x % 3u);
        x /= 3u;
    }
}

static long double tri_path(const orc_option *o, double pd, const int *dg)
{
    double pm = 1.0 - o->p - pd;
    double S = o->S, w = 1.0, sum = 0.0, mx = -INFINITY, mn = INFINITY;
    int lev = 0;
    for (int t = 0; t < o->N; ++t) {
        lev += dg[t] - 1;
        S = o->S * pow(o->u, (double)lev);
        w *= dg[t] == 2 ? o->p : (dg[t] == 1 ? pm : pd);
        sum += S;
        if (S > mx) mx = S;
        if (S < mn) mn = S;
    }
    return (long double)w *
           (long double)payoff_from_stats(o->payoff, o->K, sum, mx, mn, S, o->N);
}

double orc_price_tri_naive(const orc_option *o, double pd)
{
    if (!tri_ok(o, pd) || o->N > 18) return NAN;
    uint64_t n = 1;
    for (int t = 0; t < o->N; ++t) n *= 3u;
    int dg[64];
    ksum_t acc = {0.0L, 0.0L};
    for (uint64_t x = 0; x < n; ++x) {
        orc_tri_digits(x, o->N, dg);
        ksum_add(&acc, tri_path(o, pd, dg));
    }
    return (double)((long double)exp(-o->r * o->T) * ksum_get(&acc));
}

/* Depth-first over the tree with a table of u^l; ranks = the 3^depth
 * prefixes of the first min(N, 6) steps, combined pairwise in order. */
typedef struct {
    const orc_option *o;
    double pd, pm;
    const double *upow; /* upow[l + N] = u^l */
} tri_ctx;

static long double tri_node(const tri_ctx *c, int t, int lev, double w, double sum,
                            double mx, double mn, double last)
{
    const orc_option *o = c->o;
    if (t == o->N)
        return (long double)w *
               (long double)payoff_from_stats(o->payoff, o->K, sum, mx, mn, last, o->N);
    long double acc = 0.0L;
    for (int d = 0; d <= 2; ++d) {
        double pw = d == 2 ? o->p : (d == 1 ? c->pm : c->pd);
        if (pw == 0.0) continue;
        int l1 = lev + d - 1;
        double St = o->S * c->upow[l1 + o->N];
        acc += tri_node(c, t + 1, l1, w * pw, sum + St, St > mx ? St : mx, St < mn ? St : mn, St);
    }
    return acc;
}

typedef struct {
    const tri_ctx *c;
    int depth;
    uint64_t first, count;
    long double *out;
} tri_job;

static void *tri_worker(void *arg)
{
    tri_job *j = (tri_job *)arg;
    const tri_ctx *c = j->c;
    const orc_option *o = c->o;
    int dg[64];
    for (uint64_t z = j->first; z < j->first + j->count; ++z) {
        orc_tri_digits(z, j->depth, dg);
        int lev = 0;
        double w = 1.0, sum = 0.0, mx = -INFINITY, mn = INFINITY, last = o->S;
        for (int t = 0; t < j->depth; ++t) {
            lev += dg[t] - 1;
            last = o->S * c->upow[lev + o->N];
            w *= dg[t] == 2 ? o->p : (dg[t] == 1 ? c->pm : c->pd);
            sum += last;
            if (last > mx) mx = last;
            if (last < mn) mn = last;
        }
        j->out[z] = w == 0.0 ? 0.0L : tri_node(c, j->depth, lev, w, sum, mx, mn, last);
    }
    return NULL;
}

double orc_price_tri(const orc_option *o, double pd, int threads)
{
    if (!tri_ok(o, pd)) return NAN;
    int N = o->N;
    double *upow = (double *)malloc(sizeof(double) * (size_t)(2 * N + 1));
    if (!upow) return NAN;
    for (int l = -N; l <= N; ++l) upow[l + N] = pow(o->u, (double)l);
    tri_ctx c = {o, pd, 1.0 - o->p - pd, upow};
    int depth = N < 6 ? N : 6;
    uint64_t M = 1;
    for (int t = 0; t < depth; ++t) M *= 3u;
    long double *part = (long double *)malloc(sizeof(long double) * M);
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > M) threads = (int)M;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    tri_job *jobs = (tri_job *)malloc(sizeof(tri_job) * (size_t)threads);
    uint64_t per = M / (uint64_t)threads, extra = M % (uint64_t)threads, first = 0;
    for (int t = 0; t < threads; ++t) {
        uint64_t cnt = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (tri_job){&c, depth, first, cnt, part};
        first += cnt;
        if (threads > 1)
            pthread_create(&tid[t], NULL, tri_worker, &jobs[t]);
        else
            tri_worker(&jobs[t]);
    }
    if (threads > 1)
        for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
    long double s = pairwise(part, M);
    free(part);
    free(tid);
    free(jobs);
    free(upow);
    return (double)((long double)exp(-o->r * o->T) * s);
}

/* European payoff by backward induction on the recombining trinomial
 * lattice (levels -t..t after t steps): a textbook pin, not the method. */
double orc_tri_euro_backward(const orc_option *o, double pd)
{
    if (!tri_ok(o, pd) || (o->payoff != ORC_EURO_CALL && o->payoff != ORC_EURO_PUT)) return NAN;
    int N = o->N;
    double pm = 1.0 - o->p - pd;
    double *v = (double *)malloc(sizeof(double) * (size_t)(2 * N + 1));
    double *nv = (double *)malloc(sizeof(double) * (size_t)(2 * N + 1));
    for (int l = -N; l <= N; ++l) {
        double S = o->S * pow(o->u, (double)l);
        v[l + N] = o->payoff == ORC_EURO_CALL ? fmax(S - o->K, 0.0) : fmax(o->K - S, 0.0);
    }
    for (int t = N - 1; t >= 0; --t) {
        for (int l = -t; l <= t; ++l)
            nv[l + N] = o->p * v[l + 1 + N] + pm * v[l + N] + pd * v[l - 1 + N];
        for (int l = -t; l <= t; ++l) v[l + N] = nv[l + N];
    }
    double res = exp(-o->r * o->T) * v[N];
    free(v);
    free(nv);
    return res;
}
