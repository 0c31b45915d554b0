/*
 * bt_oracle.h -- declarations of the plain CPU reference (test
 * infrastructure only; see bt_oracle.c).  Independent of the GPU library's
 * public header: its own types, its own enumerations.
 */
#ifndef BT_ORACLE_H
#define BT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_ASIAN_CALL = 0,         /* max(mean(S_1..S_N) - K, 0)          */
    ORC_ASIAN_PUT = 1,          /* max(K - mean(S_1..S_N), 0)          */
    ORC_LOOKBACK_FLOAT = 2,     /* max(S_1..S_N) - S_N                 */
    ORC_LOOKBACK_FIXED_PUT = 3, /* max(K - min(S_1..S_N), 0)           */
    ORC_EURO_CALL = 4,          /* max(S_N - K, 0)                     */
    ORC_EURO_PUT = 5,           /* max(K - S_N, 0)                     */
    ORC_NPAYOFF = 6
};

enum { ORC_SCHEME_CRR = 0, ORC_SCHEME_SEYDEL = 1 };

typedef struct {
    double S, u, p, r, T, K;
    int32_t N, payoff;
} orc_option;

typedef struct {
    double theta;        /* sum_z P(D_z) thetahat_z (undiscounted)     */
    double var_plugin;   /* sum_z P(D_z)^2 s_z^2 / R_m, s_z^2 with 1/R_m */
    double var_unbiased; /* same with 1/(R_m - 1)                      */
    double second;       /* sum_z P(D_z) (1/R_m) sum_m V_zm^2: E[V^2]  */
} orc_mc_sums;

typedef struct {
    double value;        /* e^{-rT} theta_s                             */
    double var_plugin;   /* e^{-2rT} Var-hat, plug-in normalisation     */
    double var_unbiased; /* e^{-2rT} Var-hat, 1/(R_m - 1)               */
    double var_plain;    /* e^{-2rT} (second - theta^2) / (2^r R_m):    */
                         /* plain MC's variance at as many paths        */
} orc_mc_result;

typedef struct {
    double theta, var_plugin, var_unbiased, var_paper;
    double second;    /* sum_m P(D_m) (1/R_m) sum_i V_mi^2 */
    uint64_t samples; /* sum of R_m */
} orc_mc_prop;

/* Exact pieces (undiscounted): mean = E[V], var_total = Var[V],
 * within = sum_z P(D_z) Var[V | D_z], between = Var_D E[V | D],
 * within_sq = sum_z P(D_z)^2 Var[V | D_z], shared = Var_Y E[V | Y],
 * within_y = E_Y Var[V | Y] (Y = the last N - r steps). */
typedef struct {
    double mean, var_total, within, between, within_sq, shared, within_y;
} orc_strata_exact;

int orc_params(double sigma, double r, double T, int N, int scheme,
               double *u, double *p);
void orc_path_of_index(uint64_t x, int N, int *bits);
double orc_payoff_of_path(const orc_option *o, const int *bits);
double orc_prob_of_path(const orc_option *o, const int *bits);
double orc_price_naive(const orc_option *o);
double orc_range_naive(const orc_option *o, uint64_t x_begin, uint64_t x_end);
double orc_price_dfs(const orc_option *o, int threads);
double orc_subtree_sum(const orc_option *o, int depth, uint64_t z);
double orc_euro_closed(const orc_option *o);
double orc_euro_backward(const orc_option *o);
double orc_lookback_dp(const orc_option *o, double *m2);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
uint32_t orc_up_threshold(double p);
void orc_mc_suffix_bits(uint64_t seed, uint32_t stream, uint32_t z, uint32_t m,
                        int L, uint32_t thr, int *bits);
int orc_mc_stratified_range(const orc_option *o, int r, uint32_t Rm,
                            uint64_t seed, uint32_t stream, uint64_t z_begin,
                            uint64_t z_end, orc_mc_sums *out);
int orc_mc_stratified(const orc_option *o, int r, uint32_t Rm, uint64_t seed,
                      uint32_t stream, orc_mc_result *res);
int orc_exact_strata(const orc_option *o, int r, orc_strata_exact *out);
int orc_mc_proportional(const orc_option *o, int r, uint64_t R, uint64_t seed,
                        uint32_t stream, orc_mc_prop *out);
/* the same sums over strata [z_begin, z_end) only */
int orc_mc_proportional_range(const orc_option *o, int r, uint64_t R, uint64_t seed,
                              uint32_t stream, uint64_t z_begin, uint64_t z_end,
                              orc_mc_prop *out);
/* Shared-Sample: h_i = sum_z P(D_z) V(z, y_i), undiscounted, for the draws
 * i in [i_begin, i_end), into h_out[i - i_begin] */
int orc_mc_shared_draws(const orc_option *o, int r, uint64_t seed, uint32_t stream,
                        uint32_t i_begin, uint32_t i_end, double *h_out);
int orc_mc_shared(const orc_option *o, int r, uint32_t R, uint64_t seed, uint32_t stream,
                  orc_mc_sums *out);
/* Time-varying moves: u[t], p[t] for steps t = 1..N at index t-1 (o->u and
 * o->p are ignored). */
double orc_price_tv_naive(const orc_option *o, const double *u, const double *p);
double orc_price_tv(const orc_option *o, const double *u, const double *p, int threads);
/* Trinomial trees: o->u is the up factor, o->p the up probability, pd the
 * down probability (middle = 1 - o->p - pd, may be 0). */
int orc_params_trinomial(double sigma, double r, double T, int N, double lambda,
                         double *u, double *pu, double *pd);
void orc_tri_digits(uint64_t x, int N, int *digits);
double orc_price_tri_naive(const orc_option *o, double pd);
double orc_price_tri(const orc_option *o, double pd, int threads);
double orc_tri_euro_backward(const orc_option *o, double pd);

#ifdef __cplusplus
}
#endif
#endif
