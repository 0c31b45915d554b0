// Internal declarations shared by the HIP translation units of libbt.
//
// Layout of one option's exact-enumeration state in device memory
// (everything below is produced by the table kernel, on the GPU, in FP64):
//
//   prefix side, 2^P entries.  For binomial trees (ucount: the FP32 form,
//   Shared-Sample included, and FP64 exact trees) they are in "up-count
//   order": position q holds the prefix z whose up-count a is the smallest,
//   ties by increasing z (positions [goff[a], goff[a+1]) hold all prefixes
//   with a ups); otherwise (time-varying and trinomial trees, FP64
//   Shared-Sample) position q holds prefix z = q.
//     XC[q]              FP64 X_z of a binomial exact tree (ucount, FP64):
//                        c_z depends only on the up-count a, so Wg[a] =
//                        W_a c_a carries it
//     XC[2q], XC[2q+1]   FP64 {X_z, c_z} interleaved, one 16-byte record
//                        (time-varying and trinomial trees, Shared-Sample)
//     XG[q]              FP32 X_z - Cg[a] for the compensated FP32 path of a
//                        binomial tree (xonly): c_z depends only on the
//                        up-count a, so Wg[a] = W_a c_a carries it, in FP64;
//                        the enumeration centres the suffix operand on the
//                        same Cg[a] (see Cg)
//     XG[2q], XG[2q+1]   FP32 {X_z, g_z} for the FP32 path of time-varying and
//                        trinomial trees and of Shared-Sample draws
//     chunkU[c]          FP64 sum of U_z over work chunk c
//     Wg[a]              FP64 p^a (1-p)^(P-a) (exact binomial trees, xonly
//                        or FP64: times c_a)
//     Cg[a]              FP64 centre of up-count group a (xonly): the
//                        midpoint of X_z over the group's two extreme paths
//                        (all ups first, all downs first), scaled; it follows
//                        goff[] in the same sub-array
//     bnd_pre[4c..4c+3]  FP64 error-bound sums over chunk c: sum c rhoX,
//                        sum c, sum W rhoU (rhoX, rhoU: bounds on the
//                        rounding error of X_z, U_z as stored), and for
//                        xonly the largest FP64 error of X_z - Cg[a] over
//                        the chunk (0 otherwise)
//     hist[(3j + f) kHistBins + b]  (xonly with a bound) suffix job j's
//                        histogram of v = sign Y_s over kHistBins bins of
//                        [vlo, vhi]: f = 0 mass sum om_s in units of 2^-62
//                        (rounded up), f = 1 / 2 smallest / largest v as
//                        order-preserving integers (see ord_of)
//   (xonly with a bound, after the bound kernel: bnd_pre[4c] holds the
//   input-rounding part of the error bound over chunk c's paths that can
//   reach the money, in place of sum c rhoX)
//   suffix side, 2^k entries in natural order s:
//     Y[s] / Y32[s]      the per-suffix operand of the clamped difference
//     Om[s]              FP64 p^b (1-p)^(k-b), b = popcount(s)
//     E[s]               FP64 factor of the separable part of the payoff
//     bnd_suf[4j..4j+3]  FP64 error-bound sums over suffix job j: sum om rhoY,
//                        sum om |E|, sum om rhoE, sum om
//
// The payoff of path (z, s) is written as
//     f(z, s) = c_z * max(sign * (Y_s - X_z), 0)  +  U_z * E_s
// (with W_z = P(first P steps = z) folded into c_z and U_z); X and Y are
// scaled by 2^-e, c by 2^e, so that sign*(Y - X) lies in [-1, 1] and one
// clamped subtraction computes the max.  Scaling by a power of two is exact.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bt {

constexpr int kExactMaxN = 40;
constexpr int kMcMaxN = 64;
constexpr int kJ = 16;              // suffixes held per lane
constexpr int kTile = 64 * kJ;      // suffixes per work item
constexpr int kKahanRun = 32;       // FP32 FMA run length before a Kahan fold
                                    // (time-varying and trinomial trees)
constexpr int kBlock = 16;          // FP32 binomial: prefixes summed as one pairwise tree
constexpr int kRunBlocks = 7;       // FP32 binomial: trees per run before a Kahan fold
constexpr int kMaxChunk = 2048;     // prefixes staged in LDS per work item
constexpr int kWaves = 4;           // waves per enumeration workgroup
constexpr int kTriMaxN = 26;        // trinomial trees: 3^N paths
constexpr int kTriMaxPrefix = 16;   // 3^16 prefixes
constexpr int kTriMaxSuffix = 12;   // 3^12 suffixes

enum Payoff : int {
    ASIAN_CALL = 0,
    ASIAN_PUT = 1,
    LOOKBACK_FLOAT = 2,
    LOOKBACK_FIXED_PUT = 3,
    EURO_CALL = 4,
    EURO_PUT = 5,
    NPAYOFF = 6
};

struct OptDev {
    double S, u, p, K, disc;
    double center;     // subtracted from X and Y before scaling
    double scale;      // 2^e
    double inv_scale;  // 2^-e
    int32_t N, k, P, payoff;
    int32_t sign;      // +1: clamp(Y - X); -1: clamp(X - Y)
    int32_t tiles;     // ceil(2^k / kTile)
    int32_t chunk;     // prefixes per work chunk
    int32_t nchunks;   // ceil(2^P / chunk)
    int64_t npre, nsuf;
    int64_t item_begin;  // first work item (partial slot) of this option
    int64_t nitems;      // tiles * nchunks * wsplit
    int64_t bitem_begin; // first workgroup item of this option
    int64_t nbitems;     // nchunks * groups
    int32_t groups;      // ceil(tiles / kWaves)
    int32_t xa;          // XCD blocking of the rectangles: chunk blocks (0: none)
    int32_t wsplit;      // waves sharing one tile (kWaves / tiles when tiles < kWaves)
    int32_t out_index;   // slot in the plan's value array
    int32_t fp32;        // tables built for the FP32 path
    int32_t xonly;       // FP32 records hold X alone (binomial exact trees)
    int32_t ucount;      // prefixes in up-count order (binomial trees: FP32,
                         // and FP64 exact; with xonly or FP64, c_a in Wg[a])
    int32_t nsufjobs;    // suffix-table jobs of this option
    double eps_rel;      // error bound: relative part (weights, summation)
    double eps_pre;      // relative rounding error of each prefix price S_t
    double eps_suf;      // relative rounding error of each suffix multiplier
    double eY;           // xonly: bound on the FP64 error of every stored Y[s]
    double vlo, hw;      // xonly: histogram bins of v = sign Y: hist_bin(v, vlo, hw)
    int64_t chunk_begin; // first prefix chunk of this option within its plan
    double *XC;
    float *XG;
    double *Y;
    float *Y32;
    double *Om;
    double *E;
    double *chunkU;
    double *Wg;
    int64_t *goff;
    double *Cg;       // P + 1 group centres (xonly), right after goff
    double *bnd_pre;  // 4 per chunk (nullptr: no error bound, Shared-Sample)
    double *bnd_suf;  // 4 per suffix job
    uint64_t *hist;   // 3 kHistBins per suffix job (xonly with a bound; else nullptr)
    uint64_t *dbg_z;  // optional debug export (nullptr: off)
    int32_t *dbg_a;
    int32_t *dbg_b;
    // Shared-Sample Monte Carlo (nullptr persuf: exact enumeration).  The
    // suffix table then holds nsuf Philox-drawn suffixes of k steps, and the
    // enumeration writes, per prefix chunk c, part q of it (see wsplit) and
    // suffix s, the sum over those prefixes to persuf[(c * wsplit + q) * nsuf
    // + s] instead of an omega-weighted total.
    double *persuf;
    uint64_t seed;
    uint32_t stream_id;
    uint32_t thr;     // up iff Philox word < thr
    // Time-varying moves (nullptr: constant u, p): tv[t] = u_{t+1},
    // tv[N + t] = p_{t+1} for t < N.  FP32 tables then keep the natural
    // prefix order with the path weight folded into g, scaled by 2^wexp
    // (Wg[0] = 2^-wexp undoes it in FP64).
    const double *tv;
    int32_t wexp;
    // Branches per step: 2, or 3 for a trinomial tree (npre = 3^P, nsuf =
    // 3^k; digits base 3, first step most significant, 0 down, 1 middle,
    // 2 up with probabilities pd, 1 - p - pd, p).  FP32 tables then keep
    // the natural order with the weight in g, as for time-varying moves.
    int32_t base;
    double pd;
};

// Reads one word of every 64-byte line of an option's parameters at once,
// so that the scalar cache holds all of them before a short kernel uses
// the fields: each field's first read would otherwise wait for a memory
// round trip of its own, one after the other.
template <typename OPT>
__device__ __forceinline__ void warm_scalar_cache(const OPT &od)
{
    static_assert(sizeof(OPT) % 4 == 0, "whole words");
    constexpr int nw = (int)(sizeof(OPT) / 4);
    const uint32_t *w = reinterpret_cast<const uint32_t *>(&od);
    uint32_t t = w[nw - 1];
#pragma unroll
    for (int i = 0; i < nw; i += 16) t ^= w[i];
    __asm__ volatile("" ::"s"(t));
}

// Suffix histograms of the FP32 binomial error bound.
constexpr int kHistBins = 256;
constexpr double kHistFix = 0x1p62;  // fixed-point unit of a bin's mass

// Bin of value v: floor((v - vlo) hw) clamped to [0, kHistBins), a monotone
// map, so the bins' value sets are ordered (the same expression wherever a
// value or a threshold is binned).
__device__ __forceinline__ int hist_bin(double v, double vlo, double hw)
{
    const double g = (v - vlo) * hw;
    return g < 1.0 ? 0 : (g >= (double)kHistBins ? kHistBins - 1 : (int)g);
}

// Order-preserving map of a double onto an unsigned integer, and back.
__device__ __forceinline__ unsigned long long ord_of(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    return (b >> 63) ? ~b : (b | (1ull << 63));
}
__device__ __forceinline__ double of_ord(unsigned long long o)
{
    const unsigned long long b = (o >> 63) ? (o & ~(1ull << 63)) : ~o;
    return __builtin_bit_cast(double, b);
}

// One block of the table kernel.
enum TableKind : int { TAB_PREFIX = 0, TAB_SUFFIX = 1, TAB_WEIGHTS = 2 };
struct TableJob {
    int32_t opt;
    int32_t kind;
    int64_t first;  // first prefix position / suffix index
    int64_t count;
    int64_t chunk;  // prefix jobs: chunk index (first / od.chunk)
};

// Launch wrappers (defined in the .hip files).
hipError_t launch_tables(const OptDev *d_opts, const TableJob *d_jobs,
                         int njobs, int64_t entries, hipStream_t s);  // entries: sum of job counts
hipError_t launch_reset_counter(unsigned long long *d_counter, hipStream_t s);
// mode: 0 FP64, 1 FP32 with {X, g} records, 2 FP32 with X-only records.
// bound_chunks > 0 (mode 2 plans with an error bound: the plan's prefix
// chunks): that many more workgroups, after the grid's, form the
// active-path input term of the bound, one prefix chunk each.
hipError_t launch_enumerate(const OptDev *d_opts, int nopts, int64_t nbitems,
                            double *d_partial, int mode, int grid, int64_t bound_chunks,
                            hipStream_t s);
// values[out_index] = the option's value, values[n + out_index] = its
// error bound (when the plan has one).
hipError_t launch_reduce(const OptDev *d_opts, int nopts,
                         const double *d_partial, double *d_values,
                         hipStream_t s);
int enumerate_max_blocks_per_cu(int mode);

// Monte Carlo.
struct McArgs {
    double S, u, p, K, disc, N_d;
    int32_t N, r, L, payoff;
    uint32_t Rm, thr, stream_id, proportional;
    uint32_t by_count;     // proportional allocation in the lane kernel: strata
                           // taken in up-count order (see mc.hip)
    uint32_t rm_of_a[32];  // proportional allocation: R_m by stratum up-count
    uint64_t seed;
    int64_t nstrata;      // 2^r
    int64_t per_item;     // strata per work item (basic MC: samples)
    int64_t nitems;
};
// Equal allocation, basic MC (r = 0) or proportional allocation: 4 doubles
// per work item in d_partial4.
hipError_t launch_mc(const McArgs &a, int fp32, double *d_partial4,
                     unsigned long long *d_counter, int grid,
                     hipStream_t s);
// out4 = {value, var_plugin, var_unbiased, var_plain} (overwrites partials).
hipError_t launch_mc_combine(double *d_partial4, int64_t nitems, int plain, uint32_t Rm,
                             double disc, double var_scale, double paths, double *d_out4,
                             hipStream_t s);
hipError_t launch_shared_combine(double *d_persuf, int64_t nchunks, int64_t nsuf,
                                 double disc, double *d_out3, hipStream_t s);  // overwrites row 0
hipError_t launch_mc_bits(uint64_t seed, uint32_t stream_id, uint32_t z,
                          uint32_t m, int L, uint32_t thr, int32_t *d_bits,
                          hipStream_t s);
int mc_max_blocks_per_cu(int fp32);

}  // namespace bt
