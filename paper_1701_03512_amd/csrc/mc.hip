// Partitioned (prefix-stratified) Monte Carlo, Section 4.
//
// The strata are the 2^r prefixes of the first r steps (the sets B_m^N of
// Section 3), each with its exact probability P(D_z) = p^a (1-p)^(r-a)
// (eq. (mc9)); every stratum receives R_m suffix draws of L = N - r steps.
//
// Equal allocation (the setting of Theorem 1) and basic MC run
// mc_lane_kernel, and so does proportional allocation with at least 16
// draws per stratum on average: R_m = round(R P(D_m)) depends only on the
// stratum's up-count, so the kernel takes the strata in up-count order
// (position q holds the q-th stratum when they are sorted by up-count, then
// by index) and the lanes of a pass share one R_m but where two up-counts
// meet; a sample's draws still follow its stratum's index, so they are the
// same draws whatever the order.  A wavefront owns a work item of `per_item` consecutive
// strata and gives each stratum G lanes (G = 1 when the item holds 64 or
// more strata, else 64 / strata): lane (slot, sub) walks the r prefix steps
// of stratum z0 + slot once, in FP64 (P(D_z) and the payoff's prefix
// quantities), then draws the stratum's samples m = sub, sub + G, ... and
// keeps shifted running sums of their payoffs in FP64 (shift = its first
// payoff, so the variance does not cancel).  The G lanes of a stratum merge
// their (n, mean, M2) by a fixed butterfly (Chan, Golub, LeVeque), and the
// item accumulates, per stratum,
//     P(D_z) thetahat_z,  P(D_z)^2 s_z^2 / R_m (plug-in and 1/(R_m - 1)),
//     P(D_z) (s_z^2 + thetahat_z^2)
// in FP64 (eq. (mc12); eq. (mc13) first line; the last sum estimates E[V^2]
// and so the variance of plain MC with as many paths).  Basic MC (r = 0,
// one stratum) splits an item's samples over the 64 lanes and writes the
// merged (n, mean, M2).  Proportional allocation runs mc_flat_kernel, which
// lays a block's samples out stratum after stratum (below).
//
// A suffix walks eight steps per Philox block: up_bits8 gives the block's
// eight up bits as an 8-bit pattern x, and one read of an LDS table indexed
// by x gives what the block's steps add to the payoff's statistic relative
// to the block's starting level l0 -- sum_i (u^D_i - 1), max_i u^D_i or
// min_i u^D_i over the levels l0 + D_i the block visits -- and the level it
// ends on; one read of the level table gives u^l0 and u^l0 - 1.  So a block
// costs the Philox rounds, the pattern, two table reads and one or two
// multiply-adds, instead of eight reads and eight updates.  The statistic
// runs in FP32 (FP32 paths) or FP64; the tables are built from FP64 powers
// of u.
#include <algorithm>

#include "bt_internal.hpp"
#include "philox.hpp"

namespace bt {
namespace {

constexpr int kMcThreads = 256;
constexpr int kPow = kMcMaxN;  // level table offset: level l at [l + kPow]

// Prefix quantities per payoff (Pz = price after the r prefix steps):
//   Asian:          q1 = (N K - A_z)/Pz - L   (the suffix sum is kept as
//                   sum_j (u^l_j - 1), i.e. centred by L), g = Pz / N
//   floating lkbk:  q1 = M_z / Pz (0 for r = 0), g = Pz
//   fixed put:      q1 = K / Pz, q2 = m_z / Pz (+inf for r = 0), g = Pz
//   European:       q1 = K / Pz, g = Pz
__device__ inline void prefix_quant(const McArgs &a, double A, double M,
                                    double m, double Pz, bool empty,
                                    double &q1, double &q2, double &g)
{
    q2 = 0.0;
    switch (a.payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT:
        q1 = (a.N_d * a.K - A) / Pz - (double)a.L;
        g = Pz / a.N_d;
        break;
    case LOOKBACK_FLOAT:
        q1 = empty ? 0.0 : M / Pz;
        g = Pz;
        break;
    case LOOKBACK_FIXED_PUT:
        q1 = a.K / Pz;
        q2 = empty ? INFINITY : m / Pz;
        g = Pz;
        break;
    default:
        q1 = a.K / Pz;
        g = Pz;
        break;
    }
}

// Which suffix statistic a payoff needs (one kernel per kind, so a path
// step tracks only that statistic).
enum McKind : int { MK_ASIAN = 0, MK_LOOKBACK_FLOAT = 1, MK_LOOKBACK_FIXED = 2, MK_EURO = 3 };

constexpr int mc_kind(int payoff)
{
    return (payoff == ASIAN_CALL || payoff == ASIAN_PUT) ? MK_ASIAN
           : payoff == LOOKBACK_FLOAT                    ? MK_LOOKBACK_FLOAT
           : payoff == LOOKBACK_FIXED_PUT                ? MK_LOOKBACK_FIXED
                                                         : MK_EURO;
}

// Level table entry: u^l and u^l - 1 (the price relative to the prefix end
// at level l, and its centred form for the Asian sum).
// (aligned to its size, so that one LDS read at a constant offset loads it)
template <typename F>
struct __attribute__((aligned(2 * sizeof(F)))) LevE {
    F ul, um1;
};

// Block table entry for an up pattern x of the block's steps: the block's
// contribution t relative to its starting level (see the header) and the
// change of level in bytes of the level table.
template <typename F>
struct PatE {
    F t;
    int32_t dl;
};

// The walk tables of a workgroup: levels -kPow..kPow from the FP64 powers
// upd[], and two pattern tables, for full blocks of eight steps and for the
// last block's L mod 8 steps (its pattern bits above those steps are masked
// off).
template <typename F, int KIND>
__device__ void build_walk_tables(const McArgs &a, const double *upd, LevE<F> *lev,
                                  PatE<F> (*pat)[256])
{
    for (int l = threadIdx.x; l <= 2 * kPow; l += blockDim.x) {
        lev[l].ul = (F)upd[l];
        lev[l].um1 = (F)(upd[l] - 1.0);
    }
    const int rem = a.L & 7;
    for (int e = threadIdx.x; e < 512; e += blockDim.x) {
        const int which = e >> 8;
        const uint32_t x = (uint32_t)e & 255u;
        const int n = which ? rem : 8;
        int D = 0;
        double t = KIND == MK_ASIAN ? 0.0 : (KIND == MK_LOOKBACK_FLOAT ? -INFINITY : INFINITY);
        for (int i = 0; i < n; ++i) {
            D += ((x >> i) & 1u) ? 1 : -1;
            const double v = upd[D + kPow];
            if (KIND == MK_ASIAN) t += v - 1.0;
            else if (KIND == MK_LOOKBACK_FLOAT) t = fmax(t, v);
            else if (KIND == MK_LOOKBACK_FIXED) t = fmin(t, v);
        }
        pat[which][x].t = (KIND == MK_EURO || n == 0) ? (F)0 : (F)t;
        pat[which][x].dl = D * (int)sizeof(LevE<F>);
    }
}

// Fused multiply-add in the statistic's own precision.
__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One block of n steps with up pattern x, starting at the byte offset lofs
// of the level table: update the statistic and move the level.
template <typename F, int KIND>
__device__ __forceinline__ void walk_block(const char *lb, const PatE<F> *pat, uint32_t x, F n,
                                           int &lofs, F &acc)
{
    const PatE<F> e = pat[x];
    const LevE<F> lv = *reinterpret_cast<const LevE<F> *>(lb + lofs);
    if constexpr (KIND == MK_ASIAN) {
        // sum over the block of (u^(l0 + D_i) - 1) = u^l0 t + n (u^l0 - 1)
        acc = fma_of(lv.ul, e.t, acc);
        acc = fma_of(lv.um1, n, acc);
    } else if constexpr (KIND == MK_LOOKBACK_FLOAT) {
        acc = fmax(acc, lv.ul * e.t);  // one v_max (no NaN can arise)
    } else if constexpr (KIND == MK_LOOKBACK_FIXED) {
        acc = fmin(acc, lv.ul * e.t);
    }
    lofs += e.dl;
}

// One sample's payoff from its suffix draws.
template <typename F, int KIND>
__device__ __forceinline__ F sample_payoff(const McArgs &a, const LevE<F> *lev,
                                           const PatE<F> (*pat)[256], F q1, F q2, F g,
                                           uint32_t m, uint32_t z)
{
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const char *lb = reinterpret_cast<const char *>(lev);
    F acc = KIND == MK_ASIAN ? (F)0 : (KIND == MK_LOOKBACK_FLOAT ? (F)-INFINITY : (F)INFINITY);
    int lofs = kPow * (int)sizeof(LevE<F>);  // level 0: the prefix end
    const int nfull = a.L >> 3, rem = a.L & 7;
    for (int b = 0; b < nfull; ++b) {
        const uint32_t x = up_bits8((uint32_t)b, m, z, a.stream_id, k0, k1, a.thr);
        walk_block<F, KIND>(lb, pat[0], x, (F)8, lofs, acc);
    }
    if (rem) {
        const uint32_t x = up_bits8((uint32_t)nfull, m, z, a.stream_id, k0, k1, a.thr);
        walk_block<F, KIND>(lb, pat[1], x & ((1u << rem) - 1u), (F)rem, lofs, acc);
    }
    const F last = reinterpret_cast<const LevE<F> *>(lb + lofs)->ul;
    F v;
    if constexpr (KIND == MK_ASIAN) {
        v = a.payoff == ASIAN_CALL ? g * fmax(acc - q1, (F)0) : g * fmax(q1 - acc, (F)0);
    } else if constexpr (KIND == MK_LOOKBACK_FLOAT) {
        v = g * ((q1 > acc ? q1 : acc) - last);
    } else if constexpr (KIND == MK_LOOKBACK_FIXED) {
        v = g * fmax(q1 - (q2 < acc ? q2 : acc), (F)0);
    } else {
        v = a.payoff == EURO_CALL ? g * fmax(last - q1, (F)0) : g * fmax(q1 - last, (F)0);
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;  // lane 0's value is the fixed-order total
}

__device__ __forceinline__ double bcast(double v, int lane_src)
{
    return __shfl(v, lane_src);
}

// Value of a wave-uniform lane (both 32-bit halves read with v_readlane).
__device__ __forceinline__ double lane_value(double v, int lane)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A DPP move of a double (both halves with the same control); lanes of rows
// outside ROWS receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, unsigned d)
{
    const uint32_t lo = __shfl_up((uint32_t)v, d), hi = __shfl_up((uint32_t)(v >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan of x over the lanes [first, lane] of the caller's segment
// (segments are runs of consecutive lanes), with DPP moves in a fixed tree:
// shifts by 1, 2, 4 and 8 inside each 16-lane row, then lane 15 of rows 0
// and 2 into rows 1 and 3, then lane 31 into rows 2 and 3.  A lane adds a
// moved value only when its source lane lies in the same segment, so the
// order of the additions depends only on the segment layout.
__device__ __forceinline__ double seg_scan(double x, int lane, int first)
{
    const int r = lane & 15;
    double y;
    y = dpp_f64<0x111, 0xF>(x);  // row_shr:1
    if (r >= 1 && lane - 1 >= first) x += y;
    y = dpp_f64<0x112, 0xF>(x);  // row_shr:2
    if (r >= 2 && lane - 2 >= first) x += y;
    y = dpp_f64<0x114, 0xF>(x);  // row_shr:4
    if (r >= 4 && lane - 4 >= first) x += y;
    y = dpp_f64<0x118, 0xF>(x);  // row_shr:8
    if (r >= 8 && lane - 8 >= first) x += y;
    y = dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    if (((lane >> 4) & 1) && (lane & ~15) - 1 >= first) x += y;
    y = dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    if (lane >= 32 && 31 >= first) x += y;
    return x;
}

__device__ __forceinline__ int64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Work items: taken from the counter one at a time (many items: the waves
// that finish first take more), or, with no counter, cyclically by wave
// (wave w takes w, w + W, w + 2W, ... for W waves).  The cyclic form issues
// no atomics: every wave's first atomic on the one counter serialises
// across the device, a floor of about 0.1 ms under a launch of a few
// thousand items.  The result does not depend on the order: each item
// writes its own partial.
__device__ __forceinline__ int64_t next_item(unsigned long long *counter, int lane)
{
    unsigned long long v = 0;
    if (lane == 0) v = atomicAdd(counter, 1ull);
    return uniform64(v);
}

__device__ __forceinline__ int64_t first_item(unsigned long long *counter, int lane)
{
    if (counter) return next_item(counter, lane);
    return (int64_t)blockIdx.x * (blockDim.x >> 6) +
           (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ int64_t following_item(unsigned long long *counter, int lane,
                                                  int64_t item)
{
    if (counter) return next_item(counter, lane);
    return item + (int64_t)gridDim.x * (blockDim.x >> 6);
}

// FP64 powers u^l, l = -kPow..kPow, P(D_z) by the stratum's up-count, and
// the walk tables; ends with a barrier.
template <typename F, int KIND>
__device__ void setup_tables(const McArgs &a, double *upd, double *wstr, LevE<F> *lev,
                             PatE<F> (*pat)[256])
{
    for (int l = threadIdx.x; l <= 2 * kPow; l += blockDim.x) upd[l] = pow(a.u, (double)(l - kPow));
    for (int u = threadIdx.x; u <= a.r; u += blockDim.x)
        wstr[u] = pow(a.p, (double)u) * pow(1.0 - a.p, (double)(a.r - u));
    __syncthreads();
    build_walk_tables<F, KIND>(a, upd, lev, pat);
    __syncthreads();
}

// Combine (n_b, mean_b, M2_b) into (n, mean, M2): Chan, Golub, LeVeque.
__device__ __forceinline__ void chan_merge(double &n, double &mean, double &M2,
                                           double nb, double meanb, double M2b)
{
    if (nb == 0.0) return;
    if (n == 0.0) {
        n = nb; mean = meanb; M2 = M2b;
        return;
    }
    const double nn = n + nb, d = meanb - mean;
    mean += d * (nb / nn);
    M2 += M2b + d * d * (n * nb / nn);
    n = nn;
}

// Prefix state of stratum z (its first r steps, FP64): P(D_z) and the
// payoff's prefix quantities.
__device__ __forceinline__ void prefix_state(const McArgs &a, const double *upd,
                                             const double *wstr, int64_t z, double &W,
                                             double &q1, double &q2, double &g)
{
    int lev = 0, ups = 0;
    double A = 0.0, M = -INFINITY, m = INFINITY;
    for (int t = 1; t <= a.r; ++t) {
        const int bit = (int)((z >> (a.r - t)) & 1);
        ups += bit;
        lev += bit ? 1 : -1;
        const double St = a.S * upd[lev + kPow];
        A += St;
        M = fmax(M, St);
        m = fmin(m, St);
    }
    const double Pz = (a.r > 0) ? a.S * upd[lev + kPow] : a.S;
    W = wstr[ups];
    prefix_quant(a, A, M, m, Pz, a.r == 0, q1, q2, g);
}

// (n, mean, M2) of the payoffs of samples m0, m0 + step, ... < mend of
// stratum z, from running sums shifted by the first payoff.
template <typename F, int KIND>
__device__ __forceinline__ void lane_stats(const McArgs &a, const LevE<F> *lev,
                                           const PatE<F> (*pat)[256], F q1, F q2, F g,
                                           uint32_t m0, uint32_t step, uint32_t mend,
                                           uint32_t z, double &n, double &mean, double &M2)
{
    n = mean = M2 = 0.0;
    if (m0 >= mend) return;
    const double K = (double)sample_payoff<F, KIND>(a, lev, pat, q1, q2, g, m0, z);
    double s1 = 0.0, s2 = 0.0, cnt = 1.0;
    for (uint32_t m = m0 + step; m < mend; m += step) {
        const double d = (double)sample_payoff<F, KIND>(a, lev, pat, q1, q2, g, m, z) - K;
        s1 += d;
        s2 = __builtin_fma(d, d, s2);
        cnt += 1.0;
    }
    n = cnt;
    mean = K + s1 / cnt;
    M2 = fmax(s2 - s1 * (s1 / cnt), 0.0);
}

// Stratum at position q of the up-count order: the group a with goff[a] <=
// q < goff[a + 1] (goff[a] = sum_{b < a} C(r, b)), then the (q - goff[a])-th
// r-bit number with a ones in increasing order: walking the bits from the
// most significant, the C(i, rem) numbers with bit i clear come first.
constexpr int kMaxStrataSteps = 30;
__device__ __forceinline__ int64_t stratum_at(int64_t q, int r,
                                              const uint32_t (*binom)[kMaxStrataSteps + 2],
                                              const int64_t *goff, int &ups)
{
    int a = 0;
    while (goff[a + 1] <= q) ++a;
    ups = a;
    uint64_t rank = (uint64_t)(q - goff[a]);
    int rem = a;
    int64_t z = 0;
    for (int i = r - 1; i >= 0 && rem > 0; --i) {
        const uint64_t c = rem <= i ? binom[i][rem] : 0u;
        if (rank >= c) {
            z |= (int64_t)1 << i;
            rank -= c;
            --rem;
        }
    }
    return z;
}

// Binomial coefficients C(n, k), n <= r, and the group offsets of the
// up-count order (by_count launches only); ends with a barrier.
__device__ void setup_count_order(const McArgs &a, uint32_t (*binom)[kMaxStrataSteps + 2],
                                  int64_t *goff)
{
    for (int e = threadIdx.x; e < (kMaxStrataSteps + 1) * (kMaxStrataSteps + 2); e += blockDim.x) {
        const int n = e / (kMaxStrataSteps + 2), k = e % (kMaxStrataSteps + 2);
        uint64_t c = k <= n ? 1u : 0u;
        for (int j = 1; j <= k && k <= n; ++j) c = c * (uint64_t)(n - k + j) / (uint64_t)j;
        binom[n][k] = (uint32_t)c;
    }
    __syncthreads();
    for (int g = threadIdx.x; g <= a.r + 1; g += blockDim.x) {
        int64_t o = 0;
        for (int b = 0; b < g; ++b) o += binom[a.r][b];
        goff[g] = o;
    }
    __syncthreads();
}

// Equal allocation, basic MC and proportional allocation in up-count order
// (see the header).  partial4 per item: stratified {sum W theta, sum W^2
// s^2/R_m (proportional: sum of the raw M2, the 1/R^2 estimator being
// scaled in the combine), same with 1/(R_m - 1), sum W (s^2 + theta^2)};
// basic {n, mean, M2, 0}.  BYCOUNT: proportional allocation (a.by_count),
// a separate instantiation so that equal allocation keeps its uniform
// per-stratum arithmetic.
template <typename F, int KIND, bool BYCOUNT>
__global__ __launch_bounds__(kMcThreads) void mc_lane_kernel(
    const McArgs a, double *__restrict__ partial4, unsigned long long *counter)
{
    __shared__ double upd[2 * kPow + 1];
    __shared__ double wstr[kPow + 1];
    __shared__ LevE<F> lev[2 * kPow + 1];
    __shared__ PatE<F> pat[2][256];
    __shared__ uint32_t binom[BYCOUNT ? kMaxStrataSteps + 1 : 1][kMaxStrataSteps + 2];
    __shared__ int64_t goff[kMaxStrataSteps + 2];
    setup_tables<F, KIND>(a, upd, wstr, lev, pat);
    if constexpr (BYCOUNT) setup_count_order(a, binom, goff);

    const int lane = threadIdx.x & 63;
    const bool plain = a.r == 0;
    // lanes per stratum: 64 / (strata of an item), at least 1
    int64_t span = plain ? 1 : (a.per_item < a.nstrata ? a.per_item : a.nstrata);
    if (span > 64) span = 64;
    const int G = (int)(64 / span);
    const int slot = lane / G, sub = lane - slot * G;
    int64_t item = first_item(counter, lane);
    while (item < a.nitems) {
        const int64_t next = following_item(counter, lane, item);
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
        if (plain) {
            double q1, q2, g;
            prefix_quant(a, 0.0, -INFINITY, INFINITY, a.S, true, q1, q2, g);
            const uint64_t R = (uint64_t)a.Rm;
            const uint64_t mb0 = (uint64_t)item * (uint64_t)a.per_item;
            const uint64_t me = (mb0 + a.per_item < R) ? mb0 + a.per_item : R;
            double n, mean, M2;
            lane_stats<F, KIND>(a, lev, pat, (F)q1, (F)q2, (F)g, (uint32_t)(mb0 + lane), 64u,
                                (uint32_t)me, 0u, n, mean, M2);
            for (int off = 1; off < 64; off <<= 1) {
                const double nb = __shfl_xor(n, off), mb = __shfl_xor(mean, off),
                             Mb = __shfl_xor(M2, off);
                chan_merge(n, mean, M2, nb, mb, Mb);
            }
            c0 = n;
            c1 = mean;
            c2 = M2;
        } else {
            const int64_t zb = item * a.per_item;
            const int64_t ze = (zb + a.per_item < a.nstrata) ? zb + a.per_item : a.nstrata;
            const double R = (double)a.Rm;
            for (int64_t z0 = zb; z0 < ze; z0 += 64 / G) {
                const int64_t q = z0 + slot;  // the stratum's position
                const bool act = q < ze;
                double W = 0.0, q1 = 0.0, q2 = 0.0, g = 0.0;
                double n = 0.0, mean = 0.0, M2 = 0.0;
                uint32_t Rz = a.Rm;
                if (act) {
                    if constexpr (BYCOUNT) {
                        int ups;
                        const int64_t z = stratum_at(q, a.r, binom, goff, ups);
                        Rz = a.rm_of_a[ups];
                        prefix_state(a, upd, wstr, z, W, q1, q2, g);
                        lane_stats<F, KIND>(a, lev, pat, (F)q1, (F)q2, (F)g, (uint32_t)sub,
                                            (uint32_t)G, Rz, (uint32_t)z, n, mean, M2);
                    } else {
                        // (a separate call: its draw count stays wave-uniform)
                        prefix_state(a, upd, wstr, q, W, q1, q2, g);
                        lane_stats<F, KIND>(a, lev, pat, (F)q1, (F)q2, (F)g, (uint32_t)sub,
                                            (uint32_t)G, a.Rm, (uint32_t)q, n, mean, M2);
                    }
                }
                // merge the stratum's G lanes (a fixed butterfly)
                for (int off = 1; off < G; off <<= 1) {
                    const double nb = __shfl_xor(n, off), mb = __shfl_xor(mean, off),
                                 Mb = __shfl_xor(M2, off);
                    chan_merge(n, mean, M2, nb, mb, Mb);
                }
                if (act && sub == 0) {
                    const double W2 = W * W;
                    c0 += W * mean;
                    if constexpr (BYCOUNT) {  // proportional: this stratum's R_m
                        const double Rd = (double)Rz, s2 = M2 / Rd;
                        c1 += M2;
                        if (Rz > 1) c2 += W2 * (M2 / (Rd - 1.0)) / Rd;
                        c3 += W * (s2 + mean * mean);
                    } else {
                        const double s2 = M2 / R;
                        c1 += W2 * s2 / R;
                        if (a.Rm > 1) c2 += W2 * (M2 / (R - 1.0)) / R;
                        c3 += W * (s2 + mean * mean);
                    }
                }
            }
            c0 = wave_sum(c0);
            c1 = wave_sum(c1);
            c2 = wave_sum(c2);
            c3 = wave_sum(c3);
        }
        if (lane == 0) {
            partial4[4 * item + 0] = c0;
            partial4[4 * item + 1] = c1;
            partial4[4 * item + 2] = c2;
            partial4[4 * item + 3] = c3;
        }
        item = next;
    }
}

// Proportional allocation.  A wave owns 64 consecutive strata; their samples
// are laid out stratum after stratum (R_z each) and the wave takes 64
// consecutive ones per pass, so no lane idles whatever the R_z.  Lane l's
// stratum z0 + l owns samples [st, en) of the layout (a scan over the
// lanes); a sample finds its stratum by binary search over the lanes'
// starts.  In a pass each stratum's lanes form a segment whose mean and
// squared deviations come from segmented scans; a stratum cut by the pass
// boundary carries (n, mean, M2) on to the next pass, merged in sample
// order (Chan et al.).  partial4 as for equal allocation, with the raw sum
// of M2 in place of the plug-in term (the 1/R^2 estimator is scaled in the
// combine).
template <typename F, int KIND>
__global__ __launch_bounds__(kMcThreads) __attribute__((amdgpu_waves_per_eu(5))) void mc_flat_kernel(
    const McArgs a, double *__restrict__ partial4, unsigned long long *counter)
{
    __shared__ double upd[2 * kPow + 1];
    __shared__ double wstr[kPow + 1];
    __shared__ LevE<F> lev[2 * kPow + 1];
    __shared__ PatE<F> pat[2][256];
    setup_tables<F, KIND>(a, upd, wstr, lev, pat);

    const int lane = threadIdx.x & 63;
    int64_t item = first_item(counter, lane);
    while (item < a.nitems) {
        const int64_t next = following_item(counter, lane, item);
        const int64_t zb = item * a.per_item;
        const int64_t ze = (zb + a.per_item < a.nstrata) ? zb + a.per_item : a.nstrata;
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        for (int64_t z0 = zb; z0 < ze; z0 += 64) {
            const int64_t zl = z0 + lane;
            double W = 0.0, q1 = 0.0, q2 = 0.0, g = 0.0;
            int ups = 0;
            if (zl < ze) {
                prefix_state(a, upd, wstr, zl, W, q1, q2, g);
                for (int t = 1; t <= a.r; ++t) ups += (int)((zl >> (a.r - t)) & 1);
            }
            const int nz = (int)((ze - z0 < 64) ? ze - z0 : 64);
            const uint32_t Rl = lane < nz ? a.rm_of_a[ups] : 0u;
            uint64_t en = Rl;
            for (int d = 1; d < 64; d <<= 1) {
                const uint64_t y = shfl_up64(en, (unsigned)d);
                if (lane >= d) en += y;
            }
            const uint64_t st = en - Rl;
            const uint64_t T = shfl64(en, 63);
            double cn = 0.0, cmean = 0.0, cM2 = 0.0;  // carried stratum part
            double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
            for (uint64_t p0 = 0; p0 < T; p0 += 64) {
                const uint64_t pos = p0 + (uint64_t)lane;
                const bool act = pos < T;
                int j = 0;  // last lane whose stratum starts at or before pos
                for (int step = 32; step >= 1; step >>= 1)
                    if (shfl64(st, j + step) <= pos) j += step;
                const uint64_t sj = shfl64(st, j), ej = shfl64(en, j);
                int fl = sj > p0 ? (int)(sj - p0) : 0;       // segment's lanes
                int ll = ej - p0 <= 64 ? (int)(ej - p0) - 1 : 63;
                if (!act) fl = ll = lane;
                const double Wz = __shfl(W, j);
                const F fq1 = (F)__shfl(q1, j), fq2 = (F)__shfl(q2, j);
                const F fg = (F)__shfl(g, j);
                double v = 0.0;
                if (act)
                    v = (double)sample_payoff<F, KIND>(a, lev, pat, fq1, fq2, fg,
                                                       (uint32_t)(pos - sj), (uint32_t)(z0 + j));
                const double cnt = (double)(ll - fl + 1);
                const double mean = __shfl(seg_scan(v, lane, fl), ll) / cnt;
                const double dv = act ? v - mean : 0.0;
                const double m2 = __shfl(seg_scan(dv * dv, lane, fl), ll);
                double n = cnt, mu = mean, M2 = m2;
                if (act && fl == 0 && sj < p0) {  // continues the carried stratum
                    n = cn; mu = cmean; M2 = cM2;
                    chan_merge(n, mu, M2, cnt, mean, m2);
                }
                if (act && lane == ll && ej <= p0 + 64) {  // stratum complete
                    const double Rz = (double)(ej - sj);
                    const double W2 = Wz * Wz;
                    c0 += Wz * mu;
                    c1 += M2;  // the 1/R^2 form: raw M2, scaled in the combine
                    if (ej - sj > 1) c2 += W2 * (M2 / (Rz - 1.0)) / Rz;
                    c3 += Wz * (M2 / Rz + mu * mu);
                }
                cn = lane_value(n, 63);
                cmean = lane_value(mu, 63);
                cM2 = lane_value(M2, 63);
            }
            acc0 += bcast(wave_sum(c0), 0);
            acc1 += bcast(wave_sum(c1), 0);
            acc2 += bcast(wave_sum(c2), 0);
            acc3 += bcast(wave_sum(c3), 0);
        }
        if (lane == 0) {
            partial4[4 * item + 0] = acc0;
            partial4[4 * item + 1] = acc1;
            partial4[4 * item + 2] = acc2;
            partial4[4 * item + 3] = acc3;
        }
        item = next;
    }
}

// Final combine in two fixed-order stages.  Stage 1: workgroup b (one wave)
// folds the partials of items [b per, (b + 1) per) and writes the result
// over the first of them (the wave has read its whole range by then).
// Stage 2: one wave folds the nb stage-1 results (stride per).  Stratified:
// sums of the four partials.  Plain: Chan merge of (n, mean, M2).
// out4 = {value, var_plugin, var_unbiased, var_plain}, discounted; var_plain
// (stratified) = (sum W (s^2 + theta^2) - theta_s^2) / paths, the variance
// of plain MC with the same number of paths, estimated from the same draws.
__device__ __forceinline__ void fold_items(const double *__restrict__ p4, int64_t first,
                                           int64_t count, int64_t stride, int plain,
                                           double (&o)[4])
{
    const int lane = threadIdx.x;
    if (!plain) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i = lane; i < count; i += 64) {
            const double *q = p4 + 4 * (first + i * stride);
#pragma unroll
            for (int k = 0; k < 4; ++k) s[k] += q[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = wave_sum(s[k]);
        return;
    }
    double n = 0.0, mean = 0.0, M2 = 0.0;
    for (int64_t i = lane; i < count; i += 64) {
        const double *q = p4 + 4 * (first + i * stride);
        chan_merge(n, mean, M2, q[0], q[1], q[2]);
    }
    for (int off = 1; off < 64; off <<= 1) {
        const double nb = __shfl_down(n, off), mb = __shfl_down(mean, off),
                     Mb = __shfl_down(M2, off);
        if ((lane & (2 * off - 1)) == 0 && lane + off < 64) chan_merge(n, mean, M2, nb, mb, Mb);
    }
    o[0] = n;
    o[1] = mean;
    o[2] = M2;
    o[3] = 0.0;
}

__global__ __launch_bounds__(64) void mc_fold_kernel(double *__restrict__ p4, int64_t nitems,
                                                     int64_t per, int plain)
{
    const int64_t first = (int64_t)blockIdx.x * per;
    const int64_t count = (first + per < nitems ? first + per : nitems) - first;
    double o[4];
    fold_items(p4, first, count, 1, plain, o);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) p4[4 * first + k] = o[k];
}

__global__ __launch_bounds__(64) void mc_combine_kernel(
    const double *__restrict__ p4, int64_t nb, int64_t stride, int plain, double Rm,
    double disc, double var_scale, double paths, double *__restrict__ out4)
{
    double o[4];
    fold_items(p4, 0, nb, stride, plain, o);
    if (threadIdx.x != 0) return;
    const double d2 = disc * disc;
    if (!plain) {
        out4[0] = disc * o[0];
        out4[1] = d2 * (o[1] * var_scale);
        out4[2] = (Rm > 1.0) ? d2 * o[2] : NAN;
        out4[3] = d2 * fmax(o[3] - o[0] * o[0], 0.0) / paths;
        return;
    }
    out4[0] = disc * o[1];
    out4[1] = d2 * (o[2] / o[0]) / o[0];
    out4[2] = (o[0] > 1.0) ? d2 * (o[2] / (o[0] - 1.0)) / o[0] : NAN;
    out4[3] = out4[1];
}

// Shared-Sample combine.  First h_s = sum_c persuf[c * nsuf + s] over the
// rows (prefix parts) in a fixed two-level order, written over row 0 (each
// partial sum is written by the only thread that reads its inputs).  Then
// one workgroup: thetatilde = mean of h,
// Var-hat = sum (h - mean)^2 / nsuf^2 (and / (nsuf (nsuf - 1))); two passes,
// fixed-order trees.
constexpr int kCombThreads = 256;

constexpr int kRowGroup = 16;

// Stage 1: workgroup (column block, row group) sums rows [16 q, 16 q + 16)
// of its columns into row 16 q.  Stage 2: one thread per column sums rows
// 0, 16, 32, ... in order into row 0.
__global__ __launch_bounds__(kCombThreads) void shared_rowsum_kernel(
    double *__restrict__ persuf, int64_t nrows, int64_t nsuf, int64_t ncolblocks)
{
    const int64_t q = (int64_t)blockIdx.x / ncolblocks;
    const int64_t s = ((int64_t)blockIdx.x - q * ncolblocks) * kCombThreads + threadIdx.x;
    if (s >= nsuf) return;
    const int64_t r0 = q * kRowGroup;
    const int64_t r1 = (r0 + kRowGroup < nrows) ? r0 + kRowGroup : nrows;
    double h = 0.0;
    for (int64_t c = r0; c < r1; ++c) h += persuf[c * nsuf + s];
    persuf[r0 * nsuf + s] = h;
}

__global__ __launch_bounds__(kCombThreads) void shared_rowgroups_kernel(
    double *__restrict__ persuf, int64_t nrows, int64_t nsuf)
{
    const int64_t s = (int64_t)blockIdx.x * kCombThreads + threadIdx.x;
    if (s >= nsuf) return;
    double h = 0.0;
    for (int64_t c = 0; c < nrows; c += kRowGroup) h += persuf[c * nsuf + s];
    persuf[s] = h;
}

__device__ double block_sum(double v, double *red)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kCombThreads / 64; ++w) t += red[w];
    return t;
}

__global__ __launch_bounds__(kCombThreads) void shared_combine_kernel(
    const double *__restrict__ h, int64_t nsuf, double disc, double *__restrict__ out3)
{
    __shared__ double red[kCombThreads / 64];
    double s1 = 0.0;
    for (int64_t s = threadIdx.x; s < nsuf; s += kCombThreads) s1 += h[s];
    const double mean = block_sum(s1, red) / (double)nsuf;
    double s2 = 0.0;
    for (int64_t s = threadIdx.x; s < nsuf; s += kCombThreads) s2 += (h[s] - mean) * (h[s] - mean);
    const double ss = block_sum(s2, red);
    if (threadIdx.x == 0) {
        const double R = (double)nsuf;
        out3[0] = disc * mean;
        out3[1] = disc * disc * ss / (R * R);
        out3[2] = nsuf > 1 ? disc * disc * ss / (R * (R - 1.0)) : NAN;
    }
}

// Debug export: the up bits of the suffix of sample m in stratum z, as the
// walk draws them (up_bits8, eight steps per block).
__global__ void mc_bits_kernel(uint64_t seed, uint32_t stream_id, uint32_t z,
                               uint32_t m, int L, uint32_t thr, int32_t *bits)
{
    const int j = threadIdx.x;
    if (j >= L) return;
    const uint32_t x = up_bits8((uint32_t)(j >> 3), m, z, stream_id, (uint32_t)seed,
                                (uint32_t)(seed >> 32), thr);
    bits[j] = (int32_t)((x >> (j & 7)) & 1u);
}

}  // namespace

template <typename F, int KIND>
static void launch_kind(const McArgs &a, double *d_partial4, unsigned long long *d_counter,
                        int grid, hipStream_t s)
{
    // the flat kernel shares the persistent grid sized for the lane kernel:
    // any workgroups beyond its residency start as others exit and find the
    // work counter drained or nearly so
    if (a.proportional && !a.by_count)
        hipLaunchKernelGGL((mc_flat_kernel<F, KIND>), dim3(grid), dim3(kMcThreads), 0, s, a,
                           d_partial4, d_counter);
    else if (a.by_count)
        hipLaunchKernelGGL((mc_lane_kernel<F, KIND, true>), dim3(grid), dim3(kMcThreads), 0, s, a,
                           d_partial4, d_counter);
    else
        hipLaunchKernelGGL((mc_lane_kernel<F, KIND, false>), dim3(grid), dim3(kMcThreads), 0, s, a,
                           d_partial4, d_counter);
}

template <typename F>
static void launch_typed(const McArgs &a, double *d_partial4, unsigned long long *d_counter,
                         int grid, hipStream_t s)
{
    switch (mc_kind(a.payoff)) {
    case MK_ASIAN: launch_kind<F, MK_ASIAN>(a, d_partial4, d_counter, grid, s); break;
    case MK_LOOKBACK_FLOAT: launch_kind<F, MK_LOOKBACK_FLOAT>(a, d_partial4, d_counter, grid, s); break;
    case MK_LOOKBACK_FIXED: launch_kind<F, MK_LOOKBACK_FIXED>(a, d_partial4, d_counter, grid, s); break;
    default: launch_kind<F, MK_EURO>(a, d_partial4, d_counter, grid, s); break;
    }
}

hipError_t launch_mc(const McArgs &a, int fp32, double *d_partial4,
                     unsigned long long *d_counter, int grid, hipStream_t s)
{
    if (fp32)
        launch_typed<float>(a, d_partial4, d_counter, grid, s);
    else
        launch_typed<double>(a, d_partial4, d_counter, grid, s);
    return hipGetLastError();
}

hipError_t launch_mc_combine(double *d_partial4, int64_t nitems, int plain,
                             uint32_t Rm, double disc, double var_scale, double paths,
                             double *d_out4, hipStream_t s)
{
    if (nitems < 1) return hipErrorInvalidValue;
    // at most 1024 stage-1 groups of at least 256 items
    int64_t per = (nitems + 1023) / 1024;
    if (per < 256) per = 256;
    const int64_t nb = (nitems + per - 1) / per;
    hipLaunchKernelGGL(mc_fold_kernel, dim3((unsigned)nb), dim3(64), 0, s, d_partial4, nitems,
                       per, plain);
    hipLaunchKernelGGL(mc_combine_kernel, dim3(1), dim3(64), 0, s, (const double *)d_partial4,
                       nb, per, plain, (double)Rm, disc, var_scale, paths, d_out4);
    return hipGetLastError();
}

hipError_t launch_shared_combine(double *d_persuf, int64_t nchunks, int64_t nsuf,
                                 double disc, double *d_out3, hipStream_t s)
{
    if (nchunks < 1 || nsuf < 1) return hipErrorInvalidValue;
    const int64_t ncolblocks = (nsuf + kCombThreads - 1) / kCombThreads;
    const int64_t ngroups = (nchunks + kRowGroup - 1) / kRowGroup;
    hipLaunchKernelGGL(shared_rowsum_kernel, dim3((unsigned)(ncolblocks * ngroups)),
                       dim3(kCombThreads), 0, s, d_persuf, nchunks, nsuf, ncolblocks);
    hipLaunchKernelGGL(shared_rowgroups_kernel, dim3((unsigned)ncolblocks), dim3(kCombThreads), 0,
                       s, d_persuf, nchunks, nsuf);
    hipLaunchKernelGGL(shared_combine_kernel, dim3(1), dim3(kCombThreads), 0, s,
                       (const double *)d_persuf, nsuf, disc, d_out3);
    return hipGetLastError();
}

hipError_t launch_mc_bits(uint64_t seed, uint32_t stream_id, uint32_t z,
                          uint32_t m, int L, uint32_t thr, int32_t *d_bits,
                          hipStream_t s)
{
    hipLaunchKernelGGL(mc_bits_kernel, dim3(1), dim3(64), 0, s, seed, stream_id,
                       z, m, L, thr, d_bits);
    return hipGetLastError();
}

template <typename F>
static int min_blocks_per_cu()
{
    const void *ks[] = {
        reinterpret_cast<const void *>(mc_lane_kernel<F, MK_ASIAN, false>),
        reinterpret_cast<const void *>(mc_lane_kernel<F, MK_LOOKBACK_FLOAT, false>),
        reinterpret_cast<const void *>(mc_lane_kernel<F, MK_LOOKBACK_FIXED, false>),
        reinterpret_cast<const void *>(mc_lane_kernel<F, MK_EURO, false>)};
    int best = 0;
    for (const void *k : ks) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kMcThreads, 0) != hipSuccess ||
            nb < 1)
            return 1;
        best = best ? std::min(best, nb) : nb;
    }
    return best;
}

// Resident workgroups per CU for every lane kernel of the precision (the
// smallest over the payoff kinds), used to size the persistent grid.
int mc_max_blocks_per_cu(int fp32)
{
    return fp32 ? min_blocks_per_cu<float>() : min_blocks_per_cu<double>();
}

}  // namespace bt
