// Partitioned (prefix-stratified) Monte Carlo, Section 4.
//
// The strata are the 2^r prefixes of the first r steps (the sets B_m^N of
// Section 3), each with its exact probability P(D_z) = p^a (1-p)^(r-a)
// (eq. (mc9)); every stratum receives R_m suffix draws of L = N - r steps.
// A wavefront owns a work item of `per_item` consecutive strata:
//   1. lane l walks the r prefix steps of stratum z0 + l once (FP64), giving
//      P(D_z) and the payoff's prefix quantities;
//   2. for each stratum of the item, the quantities are broadcast from their
//      lane, lanes take samples m = lane, lane + 64, ... and walk their
//      suffix with Philox4x32-10 draws (key = seed; step j reads a 16-bit
//      half of the block with counter (j/8, m, z, stream), exact against
//      floor(p 2^32) through a fallback draw on ties; see step_keys8);
//   3. the stratum mean and the sum of squared deviations come from
//      fixed-order DPP reductions over the lanes (groups of 64 samples
//      combined in order); fewer than 64 draws per stratum share a pass
//      in lane segments, and proportional allocation lays the samples out
//      flat (mc_flat_kernel);
//   4. the item accumulates sum P(D_z) thetahat_z and
//      sum P(D_z)^2 s_z^2 / R_m (plug-in and 1/(R_m - 1) forms) in FP64 and
//      writes them to its partial slot (eq. (mc12), eq. (mc13) first line).
// Basic MC (r = 0, one stratum) splits the samples over work items instead;
// each item keeps (n, mean, M2) and the items are merged in index order with
// the pairwise update of Chan, Golub and LeVeque.
//
// The suffix walk runs in FP32 (FP32 paths) or FP64; prices come from a
// table of u^l (one rounding each), never from repeated multiplication.
#include <algorithm>

#include "bt_internal.hpp"
#include "philox.hpp"

namespace bt {
namespace {

constexpr int kMcThreads = 256;
constexpr int kPow = kMcMaxN;  // table index offset: u^l at [l + kPow]

template <typename F>
struct Quant {
    F q1, q2, g;  // payoff's prefix quantities (see prefix_quant)
};

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

// off + (bit << S) in one VALU instruction (the compiler otherwise spends a
// shift, a mask and an add on it).  Plain VALU arithmetic, no memory access.
template <int S>
__device__ __forceinline__ int lshl_add(uint32_t bit, int off)
{
    int r;
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(bit), "i"(S), "v"(off));
    return r;
}

// The statistic of one suffix step: the centred sum (Asian), or the
// running maximum (floating lookback) or minimum (fixed lookback).
template <typename F, int KIND>
__device__ __forceinline__ void take(F x, F &acc)
{
    if constexpr (KIND == MK_ASIAN) {
        acc += x;
    } else if constexpr (KIND == MK_LOOKBACK_FLOAT) {
        acc = x > acc ? x : acc;
    } else if constexpr (KIND == MK_LOOKBACK_FIXED) {
        acc = x < acc ? x : acc;
    }
}

// One sample's payoff from its suffix draws (eight steps per Philox block,
// step_keys8).  Step j with ups_j up-moves so far ends on level
// 2 ups_j - (j + 1), the table entry kPow - 1 - j + 2 ups_j.  The walk keeps
// one byte offset: 2 ups entries plus the entry of the block's last step
// (kPow - 8 - 8 b); step i of the block reads 7 - i entries further on, an
// immediate offset, so a step costs its sign bit, one shift-add and the
// read.
template <typename F, int KIND>
__device__ __forceinline__ F sample_payoff(const McArgs &a, const F *upw,
                                           const F *upm1, F q1, F q2, F g,
                                           uint32_t m, uint32_t z)
{
    constexpr int E = (int)sizeof(F);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const char *tb = reinterpret_cast<const char *>(KIND == MK_ASIAN ? upm1 : upw);
    F acc = KIND == MK_ASIAN ? (F)0 : (KIND == MK_LOOKBACK_FLOAT ? (F)-INFINITY : (F)INFINITY);
    const int nfull = a.L >> 3, rem = a.L & 7;
    int off = (kPow - 8) * E;
    int32_t key[8];
    for (int b = 0; b < nfull; ++b) {
        step_keys8((uint32_t)b, 8, m, z, a.stream_id, k0, k1, a.thr, key);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            off = lshl_add<E == 8 ? 4 : 3>((uint32_t)key[i] >> 31, off);
            if constexpr (KIND != MK_EURO)
                take<F, KIND>(*reinterpret_cast<const F *>(tb + off + (7 - i) * E), acc);
        }
        off -= 8 * E;
    }
    if (rem) {
        step_keys8((uint32_t)nfull, rem, m, z, a.stream_id, k0, k1, a.thr, key);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            if (i < rem) {
                off = lshl_add<E == 8 ? 4 : 3>((uint32_t)key[i] >> 31, off);
                if constexpr (KIND != MK_EURO)
                    take<F, KIND>(*reinterpret_cast<const F *>(tb + off + (7 - i) * E), acc);
            }
        off -= 8 * E;
    }
    // the offset left after ceil(L/8) blocks is (kPow - 8 - 8 blocks) + 2 ups entries
    const int blocks = nfull + (rem ? 1 : 0);
    const int ups = (off / E - (kPow - 8 - 8 * blocks)) >> 1;
    const F last = upw[kPow + 2 * ups - a.L];
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

// Sum over aligned segments of S lanes (S a power of two up to 64), every
// lane of a segment receiving the same total: DPP butterflies up to 16 lanes
// (quad permutes pair lane ^ 1 and lane ^ 2; the half-row and row mirrors
// pair the same partial sums as lane ^ 4 and lane ^ 8), LDS permutes above.
__device__ __forceinline__ double seg_total(double s, int S)
{
    if (S >= 2) s += dpp_f64<0xB1, 0xF>(s);
    if (S >= 4) s += dpp_f64<0x4E, 0xF>(s);
    if (S >= 8) s += dpp_f64<0x141, 0xF>(s);
    if (S >= 16) s += dpp_f64<0x140, 0xF>(s);
    for (int off = 16; off < S; off <<= 1) s += __shfl_xor(s, off);
    return s;
}

// Sum over the 64 lanes in a fixed order, returned to every lane: pairs and
// quads (quad permutes), eights and sixteens (half-row and row mirrors),
// then row 0 into row 1 and row 2 into row 3 (broadcast of lane 15 of each
// row), then rows 0-1 into rows 2-3 (broadcast of lane 31); lane 63 holds
// the total.  DPP moves only, no LDS traffic.
__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);  // row_mirror
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
    return lane_value(v, 63);
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

template <typename F>
__device__ void fill_tables(const McArgs &a, double *upd, F *upw, F *upm1)
{
    for (int l = threadIdx.x; l <= 2 * kPow; l += blockDim.x) {
        const double v = pow(a.u, (double)(l - kPow));
        upd[l] = v;
        upw[l] = (F)v;
        upm1[l] = (F)(v - 1.0);
    }
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

// The stratified estimator.  FLAT selects the flat sample layout (below),
// used for proportional allocation and for R_m above 64 that is not a
// multiple of 64, where per-stratum groups of 64 draws would leave lanes
// idle; it is a kernel of its own because it needs more registers.
template <typename F, int KIND, bool FLAT>
__device__ __forceinline__ void strat_body(const McArgs &a, double *__restrict__ partial3,
                                           unsigned long long *counter)
{
    __shared__ double upd[2 * kPow + 1];
    __shared__ F upw[2 * kPow + 1];
    __shared__ F upm1[2 * kPow + 1];
    __shared__ double wstr[kPow + 1];  // P(D_z) by the stratum's up-count
    for (int u = threadIdx.x; u <= a.r; u += blockDim.x)
        wstr[u] = pow(a.p, (double)u) * pow(1.0 - a.p, (double)(a.r - u));
    fill_tables<F>(a, upd, upw, upm1);  // ends with a barrier

    const int lane = threadIdx.x & 63;
    int64_t item = first_item(counter, lane);
    while (item < a.nitems) {
        const int64_t next = following_item(counter, lane, item);
        const int64_t zb = item * a.per_item;
        const int64_t ze = (zb + a.per_item < a.nstrata) ? zb + a.per_item : a.nstrata;
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        for (int64_t z0 = zb; z0 < ze; z0 += 64) {
            // 1. prefix state of stratum z0 + lane
            const int64_t zl = z0 + lane;
            double W = 0.0, q1 = 0.0, q2 = 0.0, g = 0.0;
            int ups = 0;
            if (zl < ze) {
                int lev = 0;
                double A = 0.0, M = -INFINITY, m = INFINITY;
                for (int t = 1; t <= a.r; ++t) {
                    const int bit = (int)((zl >> (a.r - t)) & 1);
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
            const int nz = (int)((ze - z0 < 64) ? ze - z0 : 64);
            if constexpr (FLAT) {
                // The block's samples are laid out stratum after stratum
                // (R_z each) and the wave takes 64 consecutive ones per pass,
                // so no lane idles whatever the R_z.  Lane l's stratum z0 + l
                // owns samples [st, en) of the layout (a scan over the lanes);
                // a sample finds its stratum by binary search over the lanes'
                // starts.  In a pass each stratum's lanes form a segment whose
                // mean and squared deviations come from segmented scans; a
                // stratum cut by the pass boundary carries (n, mean, M2) on to
                // the next pass, merged in sample order (Chan et al.).
                const uint32_t Rl =
                    lane < nz ? (a.proportional ? a.rm_of_a[ups] : a.Rm) : 0u;
                uint64_t en = Rl;
                for (int d = 1; d < 64; d <<= 1) {
                    const uint64_t y = shfl_up64(en, (unsigned)d);
                    if (lane >= d) en += y;
                }
                const uint64_t st = en - Rl;
                const uint64_t T = shfl64(en, 63);
                double cn = 0.0, cmean = 0.0, cM2 = 0.0;  // carried stratum part
                double c0 = 0.0, c1 = 0.0, c2 = 0.0;
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
                        v = (double)sample_payoff<F, KIND>(a, upw, upm1, fq1, fq2, fg,
                                                           (uint32_t)(pos - sj),
                                                           (uint32_t)(z0 + j));
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
                        // proportional allocation: the 1/R^2 form, a sum of
                        // raw M2 (scaled in the combine); else W^2 s^2 / R_m
                        c1 += a.proportional ? M2 : W2 * (M2 / Rz) / Rz;
                        if (ej - sj > 1) c2 += W2 * (M2 / (Rz - 1.0)) / Rz;
                    }
                    cn = lane_value(n, 63);
                    cmean = lane_value(mu, 63);
                    cM2 = lane_value(M2, 63);
                }
                acc0 += bcast(wave_sum(c0), 0);
                acc1 += bcast(wave_sum(c1), 0);
                acc2 += bcast(wave_sum(c2), 0);
                continue;
            } else if (a.seg) {
                // R_m < 64 draws per stratum: the wave takes 64 / seg strata
                // at a time, lane = (stratum slot, sample), seg lanes per
                // stratum; mean and squared deviations by fixed butterflies
                // inside the segment (every lane of it gets the same total).
                const int S = (int)a.seg, G = 64 / S;
                const int li = lane / S, ms = lane - li * S;
                const double invR = 1.0 / (double)a.Rm;
                const double invR1 = a.Rm > 1 ? 1.0 / ((double)a.Rm - 1.0) : 0.0;
                double c0 = 0.0, c1 = 0.0, c2 = 0.0;
                for (int p0 = 0; p0 < nz; p0 += G) {
                    const int zi = p0 + li;
                    const bool zact = zi < nz;
                    const int src = zact ? zi : 0;
                    const double Wz = __shfl(W, src);
                    const F fq1 = (F)__shfl(q1, src), fq2 = (F)__shfl(q2, src);
                    const F fg = (F)__shfl(g, src);
                    const bool act = zact && ms < (int)a.Rm;
                    double v = 0.0;
                    if (act)
                        v = (double)sample_payoff<F, KIND>(a, upw, upm1, fq1, fq2, fg, (uint32_t)ms,
                                                           (uint32_t)(z0 + zi));
                    const double mean = seg_total(v, S) * invR;
                    const double dv = act ? v - mean : 0.0;
                    const double s2 = seg_total(dv * dv, S);
                    if (ms == 0 && zact) {
                        const double W2 = Wz * Wz;
                        c0 += Wz * mean;
                        c1 += W2 * (s2 * invR) * invR;
                        c2 += W2 * (s2 * invR1) * invR;
                    }
                }
                acc0 += bcast(wave_sum(c0), 0);
                acc1 += bcast(wave_sum(c1), 0);
                acc2 += bcast(wave_sum(c2), 0);
                continue;
            }
            // equal allocation with R_m a multiple of 64 (or 64 or less)
            const uint32_t Rz = a.Rm;
            const double invR = 1.0 / (double)Rz;
            const double invR1 = Rz > 1 ? 1.0 / ((double)Rz - 1.0) : 0.0;
            for (int zi = 0; zi < nz; ++zi) {
                const double Wz = lane_value(W, zi);
                const F fq1 = (F)lane_value(q1, zi), fq2 = (F)lane_value(q2, zi);
                const F fg = (F)lane_value(g, zi);
                const uint32_t z = (uint32_t)(z0 + zi);
                // 2-3. samples in groups of 64, each group two-pass, groups
                // merged in order.
                double n = 0.0, mean = 0.0, M2 = 0.0;
                for (uint32_t mb = 0; mb < Rz; mb += 64) {
                    const uint32_t m = mb + (uint32_t)lane;
                    const bool act = m < Rz;
                    double v = 0.0;
                    if (act)
                        v = (double)sample_payoff<F, KIND>(a, upw, upm1, fq1, fq2, fg, m, z);
                    const uint32_t ci = (Rz - mb < 64) ? Rz - mb : 64;
                    const double cnt = (double)ci;
                    const double gmean = wave_total(v) * (ci == 64 ? 0.015625 : 1.0 / cnt);
                    const double dv = act ? v - gmean : 0.0;
                    const double gM2 = wave_total(dv * dv);
                    chan_merge(n, mean, M2, cnt, gmean, gM2);
                }
                acc0 += Wz * mean;
                const double W2 = Wz * Wz;
                acc1 += W2 * (M2 * invR) * invR;
                acc2 += W2 * (M2 * invR1) * invR;
            }
        }
        if (lane == 0) {
            partial3[3 * item + 0] = acc0;
            partial3[3 * item + 1] = acc1;
            partial3[3 * item + 2] = acc2;
        }
        item = next;
    }
}

template <typename F, int KIND>
__global__ __launch_bounds__(kMcThreads) void mc_strat_kernel(
    const McArgs a, double *__restrict__ partial3, unsigned long long *counter)
{
    strat_body<F, KIND, false>(a, partial3, counter);
}

template <typename F, int KIND>
__global__ __launch_bounds__(kMcThreads) __attribute__((amdgpu_waves_per_eu(5))) void mc_flat_kernel(
    const McArgs a, double *__restrict__ partial3, unsigned long long *counter)
{
    strat_body<F, KIND, true>(a, partial3, counter);
}

// Basic MC: one stratum (r = 0), samples [item*per_item, ...) per item;
// partial3 = (n, mean, M2).
template <typename F, int KIND>
__global__ __launch_bounds__(kMcThreads) void mc_plain_kernel(
    const McArgs a, double *__restrict__ partial3, unsigned long long *counter)
{
    __shared__ double upd[2 * kPow + 1];
    __shared__ F upw[2 * kPow + 1];
    __shared__ F upm1[2 * kPow + 1];
    fill_tables<F>(a, upd, upw, upm1);

    const int lane = threadIdx.x & 63;
    double q1, q2, g;
    prefix_quant(a, 0.0, -INFINITY, INFINITY, a.S, true, q1, q2, g);
    const F fq1 = (F)q1, fq2 = (F)q2, fg = (F)g;
    const uint64_t R = (uint64_t)a.Rm * (uint64_t)a.nstrata;  // nstrata = 1
    int64_t item = first_item(counter, lane);
    while (item < a.nitems) {
        const int64_t next = following_item(counter, lane, item);
        const uint64_t mb0 = (uint64_t)item * (uint64_t)a.per_item;
        const uint64_t me = (mb0 + a.per_item < R) ? mb0 + a.per_item : R;
        double n = 0.0, mean = 0.0, M2 = 0.0;
        for (uint64_t mb = mb0; mb < me; mb += 64) {
            const uint64_t m = mb + (uint64_t)lane;
            const bool act = m < me;
            double v = 0.0;
            if (act) v = (double)sample_payoff<F, KIND>(a, upw, upm1, fq1, fq2, fg, (uint32_t)m, 0u);
            const uint64_t ci = (me - mb < 64) ? me - mb : 64;
            const double cnt = (double)ci;
            const double gmean = wave_total(v) * (ci == 64 ? 0.015625 : 1.0 / cnt);
            const double dv = act ? v - gmean : 0.0;
            const double gM2 = wave_total(dv * dv);
            chan_merge(n, mean, M2, cnt, gmean, gM2);
        }
        if (lane == 0) {
            partial3[3 * item + 0] = n;
            partial3[3 * item + 1] = mean;
            partial3[3 * item + 2] = M2;
        }
        item = next;
    }
}

// Final combine in two fixed-order stages.  Stage 1: workgroup b (one wave)
// folds the partials of items [b per, (b + 1) per) and writes the result
// over the first of them (the wave has read its whole range by then).
// Stage 2: one wave folds the nb stage-1 results (stride per).  Stratified:
// sums of the three partials.  Plain: Chan merge of (n, mean, M2).
// out3 = {value, var_plugin, var_unbiased}, discounted.
__device__ __forceinline__ void fold_items(const double *__restrict__ p3, int64_t first,
                                           int64_t count, int64_t stride, int plain,
                                           double &o0, double &o1, double &o2)
{
    const int lane = threadIdx.x;
    if (!plain) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int64_t i = lane; i < count; i += 64) {
            const double *q = p3 + 3 * (first + i * stride);
            s0 += q[0];
            s1 += q[1];
            s2 += q[2];
        }
        o0 = wave_sum(s0);
        o1 = wave_sum(s1);
        o2 = wave_sum(s2);
        return;
    }
    double n = 0.0, mean = 0.0, M2 = 0.0;
    for (int64_t i = lane; i < count; i += 64) {
        const double *q = p3 + 3 * (first + i * stride);
        chan_merge(n, mean, M2, q[0], q[1], q[2]);
    }
    for (int off = 1; off < 64; off <<= 1) {
        const double nb = __shfl_down(n, off), mb = __shfl_down(mean, off),
                     Mb = __shfl_down(M2, off);
        if ((lane & (2 * off - 1)) == 0 && lane + off < 64) chan_merge(n, mean, M2, nb, mb, Mb);
    }
    o0 = n;
    o1 = mean;
    o2 = M2;
}

__global__ __launch_bounds__(64) void mc_fold_kernel(double *__restrict__ p3, int64_t nitems,
                                                     int64_t per, int plain)
{
    const int64_t first = (int64_t)blockIdx.x * per;
    const int64_t count = (first + per < nitems ? first + per : nitems) - first;
    double o0, o1, o2;
    fold_items(p3, first, count, 1, plain, o0, o1, o2);
    if (threadIdx.x == 0) {
        p3[3 * first + 0] = o0;
        p3[3 * first + 1] = o1;
        p3[3 * first + 2] = o2;
    }
}

__global__ __launch_bounds__(64) void mc_combine_kernel(
    const double *__restrict__ p3, int64_t nb, int64_t stride, int plain, double Rm,
    double disc, double var_scale, double *__restrict__ out3)
{
    double o0, o1, o2;
    fold_items(p3, 0, nb, stride, plain, o0, o1, o2);
    if (threadIdx.x != 0) return;
    if (!plain) {
        out3[0] = disc * o0;
        out3[1] = disc * disc * (o1 * var_scale);
        out3[2] = (Rm > 1.0) ? disc * disc * o2 : NAN;
        return;
    }
    out3[0] = disc * o1;
    out3[1] = disc * disc * (o2 / o0) / o0;
    out3[2] = (o0 > 1.0) ? disc * disc * (o2 / (o0 - 1.0)) / o0 : NAN;
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

__global__ void mc_bits_kernel(uint64_t seed, uint32_t stream_id, uint32_t z,
                               uint32_t m, int L, uint32_t thr, int32_t *bits)
{
    const int j = threadIdx.x;
    if (j >= L) return;
    int32_t key[8];
    const int b = j >> 3;
    step_keys8((uint32_t)b, L - 8 * b < 8 ? L - 8 * b : 8, m, z, stream_id, (uint32_t)seed,
               (uint32_t)(seed >> 32), thr, key);
    int32_t x = key[0];
#pragma unroll
    for (int i = 1; i < 8; ++i)
        if ((j & 7) == i) x = key[i];
    bits[j] = x < 0 ? 1 : 0;
}

}  // namespace

template <typename F, int KIND>
static void launch_kind(bool plain, const McArgs &a, double *d_partial3,
                        unsigned long long *d_counter, int grid, hipStream_t s)
{
    // the flat kernel shares the persistent grid sized for the others: any
    // workgroups beyond its residency start as others exit and find the
    // work counter drained or nearly so
    const bool flat = a.proportional || (a.seg == 0 && a.Rm > 64 && (a.Rm & 63) != 0);
    if (plain)
        hipLaunchKernelGGL((mc_plain_kernel<F, KIND>), dim3(grid), dim3(kMcThreads), 0, s, a,
                           d_partial3, d_counter);
    else if (flat)
        hipLaunchKernelGGL((mc_flat_kernel<F, KIND>), dim3(grid), dim3(kMcThreads), 0, s, a,
                           d_partial3, d_counter);
    else
        hipLaunchKernelGGL((mc_strat_kernel<F, KIND>), dim3(grid), dim3(kMcThreads), 0, s, a,
                           d_partial3, d_counter);
}

template <typename F>
static void launch_typed(bool plain, const McArgs &a, double *d_partial3,
                         unsigned long long *d_counter, int grid, hipStream_t s)
{
    switch (mc_kind(a.payoff)) {
    case MK_ASIAN: launch_kind<F, MK_ASIAN>(plain, a, d_partial3, d_counter, grid, s); break;
    case MK_LOOKBACK_FLOAT:
        launch_kind<F, MK_LOOKBACK_FLOAT>(plain, a, d_partial3, d_counter, grid, s);
        break;
    case MK_LOOKBACK_FIXED:
        launch_kind<F, MK_LOOKBACK_FIXED>(plain, a, d_partial3, d_counter, grid, s);
        break;
    default: launch_kind<F, MK_EURO>(plain, a, d_partial3, d_counter, grid, s); break;
    }
}

hipError_t launch_mc(const McArgs &a, int fp32, double *d_partial3,
                     unsigned long long *d_counter, int grid, hipStream_t s)
{
    if (fp32)
        launch_typed<float>(false, a, d_partial3, d_counter, grid, s);
    else
        launch_typed<double>(false, a, d_partial3, d_counter, grid, s);
    return hipGetLastError();
}

hipError_t launch_mc_plain(const McArgs &a, int fp32, double *d_partial3,
                           unsigned long long *d_counter, int grid, hipStream_t s)
{
    if (fp32)
        launch_typed<float>(true, a, d_partial3, d_counter, grid, s);
    else
        launch_typed<double>(true, a, d_partial3, d_counter, grid, s);
    return hipGetLastError();
}

hipError_t launch_mc_combine(double *d_partial3, int64_t nitems, int plain,
                             uint32_t Rm, double disc, double var_scale, double *d_out3,
                             hipStream_t s)
{
    if (nitems < 1) return hipErrorInvalidValue;
    // at most 1024 stage-1 groups of at least 256 items
    int64_t per = (nitems + 1023) / 1024;
    if (per < 256) per = 256;
    const int64_t nb = (nitems + per - 1) / per;
    hipLaunchKernelGGL(mc_fold_kernel, dim3((unsigned)nb), dim3(64), 0, s, d_partial3, nitems,
                       per, plain);
    hipLaunchKernelGGL(mc_combine_kernel, dim3(1), dim3(64), 0, s, (const double *)d_partial3,
                       nb, per, plain, (double)Rm, disc, var_scale, d_out3);
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
        reinterpret_cast<const void *>(mc_strat_kernel<F, MK_ASIAN>),
        reinterpret_cast<const void *>(mc_strat_kernel<F, MK_LOOKBACK_FLOAT>),
        reinterpret_cast<const void *>(mc_strat_kernel<F, MK_LOOKBACK_FIXED>),
        reinterpret_cast<const void *>(mc_strat_kernel<F, MK_EURO>),
        reinterpret_cast<const void *>(mc_plain_kernel<F, MK_ASIAN>),
        reinterpret_cast<const void *>(mc_plain_kernel<F, MK_LOOKBACK_FLOAT>),
        reinterpret_cast<const void *>(mc_plain_kernel<F, MK_LOOKBACK_FIXED>),
        reinterpret_cast<const void *>(mc_plain_kernel<F, MK_EURO>)};
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

// Resident workgroups per CU for every MC kernel of the precision (the
// smallest over the payoff kinds), used to size the persistent grid.
int mc_max_blocks_per_cu(int fp32)
{
    return fp32 ? min_blocks_per_cu<float>() : min_blocks_per_cu<double>();
}

}  // namespace bt
