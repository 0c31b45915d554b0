// Table kernel: tree quantities that every path shares, computed once.
//
//  - price multipliers u^l, l = -N..N (Section 2, A1: d = 1/u), so that the
//    price after t steps with U_t ups is S u^(2 U_t - t) (Algorithm 1 grid);
//  - path weights W_a = p^a (1-p)^(P-a) and omega_b = p^b (1-p)^(k-b): the
//    path probability p^(x'1)(1-p)^(N-x'1) of Section 2 factors into a prefix
//    part and a suffix part;
//  - prefix states (Section 3: the paths of a prefix z share their first P
//    steps, so the price at step P, the running sum, maximum and minimum are
//    computed once per prefix);
//  - suffix states: for the last k steps the sum, maximum and minimum of the
//    price multipliers relative to the prefix end, and the last multiplier
//    (for every k-step suffix, or for Philox-drawn suffixes in the
//    Shared-Sample estimator of Section 4's Remark).
//
// Trinomial trees: a path is a string of base-3 digits (down, middle, up)
// and its weight the product of the step probabilities.
//
// With time-varying moves (eq. (f13) with p_t, u_t) prices come from
// repeated multiplication by the per-step factors and weights from products
// of the per-step probabilities, for prefixes and suffixes alike.
//
// Alongside each stored X_z, U_z, Y_s and E_s the kernel bounds its
// rounding error (first-order forward analysis: every FP64 operation is
// off by at most 2^-53 of its result, every price or multiplier by the
// relative amount the host states in eps_pre / eps_suf, FP32 storage by
// 2^-24) and sums those bounds, weighted as the enumeration weights the
// quantities, into per-chunk and per-suffix-job slots.  The reduction turns
// them into the result's error bound.  Every such sum is taken over 1024
// virtual lanes in a fixed order, so it does not depend on the launch.
//
// One workgroup per job; a job is a chunk of prefix positions, a block of
// suffixes, or the per-option weight table.  All arithmetic is FP64.
#include "bt_internal.hpp"
#include "philox.hpp"

namespace bt {
namespace {

// Accesses through pointers that hold device (global) memory.  Generic
// (flat) loads and stores count against the LDS and scalar-load wait
// counter as well as the vector-memory one, so without the cast every LDS
// read of the table loops would also wait for the stores still in flight.
template <typename T>
__device__ inline __attribute__((address_space(1))) T *gm(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// The chunk sum of U is formed over kVirt virtual lanes (position i on
// lane i mod kVirt, each lane in position order, then a fixed tree), so it
// does not depend on the workgroup size the launch picks.
constexpr int kVirt = 1024;
constexpr int kVirtWaves = kVirt / 64;

__device__ inline void prefix_map(int payoff, double Nd, double K, double A,
                                  double M, double m, double Pz, bool empty,
                                  double &X, double &cf, double &U)
{
    switch (payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT:
        // mean - K = (Pz/N) (sigma_s - X) with X = (N K - A_z) / Pz
        X = (Nd * K - A) / Pz;
        cf = Pz / Nd;
        U = 0.0;
        break;
    case LOOKBACK_FLOAT: {
        // max(M_z, Pz mu_s) - Pz e_s = Pz [(mu_s - e_s) + max(M_z/Pz - mu_s, 0)]
        X = empty ? 0.0 : M / Pz;
        cf = Pz;
        U = Pz;
        break;
    }
    case LOOKBACK_FIXED_PUT: {
        // max(K - min(m_z, Pz nu_s), 0) = Pz [alpha + max(beta - nu_s, 0)]
        // with kappa = K/Pz, alpha = max(kappa - m_z/Pz, 0), beta = kappa - alpha
        double kap = K / Pz;
        double alpha = empty ? 0.0 : fmax(kap - m / Pz, 0.0);
        X = kap - alpha;
        cf = Pz;
        U = Pz * alpha;
        break;
    }
    default:  // EURO_CALL, EURO_PUT: S_N = Pz e_s
        X = K / Pz;
        cf = Pz;
        U = 0.0;
        break;
    }
}

__device__ inline void suffix_map(int payoff, double sig, double mu, double nu,
                                  double e, double &Y, double &E)
{
    switch (payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT: Y = sig; E = 0.0; break;
    case LOOKBACK_FLOAT: Y = mu; E = mu - e; break;
    case LOOKBACK_FIXED_PUT: Y = nu; E = 1.0; break;
    default: Y = e; E = 0.0; break;
    }
}

constexpr double kU64 = 0x1p-53;  // unit roundoff, FP64
constexpr double kU32 = 0x1p-24;  // unit roundoff, FP32
constexpr double kSub32 = 0x1p-149;  // FP32 rounding below the normal range

// Bounds rX, rU on the rounding error of X (before centring and scaling)
// and U as prefix_map computes them, from prices S_t (and Pz) that are each
// within a relative eS of exact, A their sum in step order (P - 1 adds).
__device__ inline void prefix_err(int payoff, double Nd, double K, double A, double m,
                                  double Pz, bool empty, int P, double eS, double X,
                                  double U, double &rX, double &rU)
{
    const double u = kU64;
    switch (payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT: {
        const double eA = eS + P * u;
        const double D = Nd * K - A;
        rX = (u * Nd * K + eA * A + u * fabs(D)) / Pz + fabs(X) * (eS + u);
        rU = 0.0;
        break;
    }
    case LOOKBACK_FLOAT:
        rX = fabs(X) * (2.0 * eS + u);
        rU = Pz * eS;
        break;
    case LOOKBACK_FIXED_PUT: {
        const double kap = K / Pz;
        const double rk = kap * (eS + u);
        if (empty) {
            rX = rk;
            rU = 0.0;
            break;
        }
        const double q = m / Pz;
        // alpha = max(kap - q, 0): where kap - q is below minus its own
        // error bound, the exact difference is negative too and both are 0
        const double rd = rk + q * (2.0 * eS + u) + u * fabs(kap - q);
        const double ra = (kap - q <= -rd) ? 0.0 : rd;
        rX = rk + ra + u * fabs(X);
        rU = Pz * ra + fabs(U) * (eS + u);
        break;
    }
    default:  // K / Pz
        rX = fabs(X) * (eS + u);
        rU = 0.0;
        break;
    }
}

// The same for Y and E as suffix_map forms them from multipliers that are
// each within a relative eM of exact, sig their sum (k - 1 adds).
__device__ inline void suffix_err(int payoff, double sig, double mu, double nu, double e,
                                  int k, double eM, double E, double &rY, double &rE)
{
    switch (payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT: rY = (eM + k * kU64) * sig; rE = 0.0; break;
    case LOOKBACK_FLOAT: rY = eM * mu; rE = eM * (mu + e) + kU64 * fabs(E); break;
    case LOOKBACK_FIXED_PUT: rY = eM * nu; rE = 0.0; break;
    default: rY = eM * e; rE = 0.0; break;
    }
}

// Multiplier c_a of the clamped term for a prefix with a ups out of P
// (constant moves): Pz = S u^(2a - P), c = Pz / N (Asian) or Pz.
__device__ inline double group_cf(const OptDev &od, const double *upow, int a)
{
    const double Pz = (od.P == 0) ? od.S : od.S * upow[2 * a - od.P + od.N];
    return (od.payoff == ASIAN_CALL || od.payoff == ASIAN_PUT) ? Pz / (double)od.N : Pz;
}

// Fixed-order sum of four per-lane values over the virtual waves of a
// workgroup: lane sums by a butterfly, then virtual wave 0, 1, ... .
__device__ inline void vsum4_lane(double (&v)[4], double (*red)[kVirtWaves], int vw, int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double x = v[i];
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) red[i][vw] = x;
    }
}

// Binomial coefficients C(n, r) for n, r <= kMaxUnrank, built at compile
// time (Pascal's rule) into constant memory.
constexpr int kMaxUnrank = 32;
struct BinomTable {
    uint64_t c[kMaxUnrank + 1][kMaxUnrank + 1];
};
constexpr BinomTable make_binom()
{
    BinomTable b{};
    for (int n = 0; n <= kMaxUnrank; ++n) {
        b.c[n][0] = 1;
        for (int r = 1; r <= n; ++r) b.c[n][r] = b.c[n - 1][r - 1] + (r <= n - 1 ? b.c[n - 1][r] : 0);
    }
    return b;
}
__constant__ BinomTable kBinom = make_binom();

// Position q -> prefix z: q - goff[a] is the rank of z among the P-bit
// numbers with a ones, in increasing order.  Walking the bits from the most
// significant, the numbers with bit i clear come first and there are C(i, r)
// of them (r = ones still to place).
__device__ inline uint64_t unrank(const uint64_t (*binom)[kMaxUnrank + 1], int64_t rank, int P,
                                  int a)
{
    uint64_t z = 0;
    int r = a;
    uint64_t rk = (uint64_t)rank;
    for (int i = P - 1; i >= 0 && r > 0; --i) {
        const uint64_t c = (r <= i) ? binom[i][r] : 0;  // C(i, r)
        if (rk >= c) {
            z |= (uint64_t)1 << i;
            rk -= c;
            --r;
        }
    }
    return z;
}

// The running quantity of the price path that a payoff needs: the sum
// (arithmetic average, Asian), the maximum (floating-strike lookback), the
// minimum (fixed-strike lookback put), or none (European: the end price).
enum Walk : int { WALK_SUM, WALK_MAX, WALK_MIN, WALK_END };

__device__ inline int walk_of(int payoff)
{
    switch (payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT: return WALK_SUM;
    case LOOKBACK_FLOAT: return WALK_MAX;
    case LOOKBACK_FIXED_PUT: return WALK_MIN;
    default: return WALK_END;
    }
}

// Constant moves: the steps of a path's `steps` bits (first step most
// significant), as multipliers upow[lev + N] of the level reached after
// each step, folded into `acc` in step order by the payoff's walk.  The
// levels follow from the bits alone, so the table reads of eight steps are
// issued together before `acc` takes them.  Returns the final level.
template <int KIND>
__device__ inline int walk_bits(uint32_t bits, int steps, int N, const double *upow, double &acc)
{
    int lev = 0;
    for (int t0 = 1; t0 <= steps; t0 += 8) {
        double m[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int t = t0 + q;
            lev += t <= steps ? 2 * (int)((bits >> (steps - t)) & 1u) - 1 : 0;
            m[q] = upow[lev + N];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (t0 + q <= steps) {
                if (KIND == WALK_SUM) acc += m[q];
                if (KIND == WALK_MAX) acc = fmax(acc, m[q]);
                if (KIND == WALK_MIN) acc = fmin(acc, m[q]);
            }
    }
    return lev;
}

// The same for a prefix, whose running sum is over prices S u^lev (the
// maximum and the minimum are taken over the multipliers and scaled once:
// S > 0 and rounding is monotone, so the result is the same).
__device__ inline int walk_prefix_sum(uint32_t bits, int steps, int N, double S,
                                      const double *upow, double &A)
{
    int lev = 0;
    for (int t0 = 1; t0 <= steps; t0 += 8) {
        double st[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int t = t0 + q;
            lev += t <= steps ? 2 * (int)((bits >> (steps - t)) & 1u) - 1 : 0;
            st[q] = S * upow[lev + N];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (t0 + q <= steps) A += st[q];
    }
    return lev;
}

template <int TH>
__global__ __launch_bounds__(TH) void table_kernel(
    const OptDev *__restrict__ opts, const TableJob *__restrict__ jobs)
{
    __shared__ double upow[2 * kMcMaxN + 1];
    __shared__ double wtab[kMcMaxN + 1];
    __shared__ double red[4][kVirtWaves];
    __shared__ uint64_t binom[kMaxUnrank][kMaxUnrank + 1];  // rows 0..P-1
    __shared__ int64_t goff[kMaxUnrank + 2];
    __shared__ double tvu[kMcMaxN], tvp[kMcMaxN];
    __shared__ uint32_t pw3[kTriMaxPrefix + 1];  // trinomial trees: 3^i (< 2^32)

    const TableJob job = jobs[blockIdx.x];
    const OptDev &od = opts[job.opt];
    warm_scalar_cache(od);
    const int N = od.N, P = od.P, k = od.k;
    const int tid = threadIdx.x;
    const bool tv = od.tv != nullptr;
    const bool tri = od.base == 3;
    const double pm = 1.0 - od.p - od.pd;  // trinomial middle probability

    // Base-3 digits: prefixes have at most kTriMaxPrefix digits and suffixes
    // kTriMaxSuffix, so positions and powers fit 32-bit integers.
    if (tri)
        for (int i = tid; i <= kTriMaxPrefix; i += TH) {
            uint32_t v = 1;
            for (int j = 0; j < i; ++j) v *= 3u;
            pw3[i] = v;
        }

    if (tv) {
        // time-varying moves: step t + 1 has factor tvu[t], probability tvp[t]
        for (int t = tid; t < N; t += TH) {
            tvu[t] = gm(od.tv)[t];
            tvp[t] = gm(od.tv)[N + t];
        }
    } else {
        for (int l = tid; l <= 2 * N; l += TH)
            upow[l] = pow(od.u, (double)(l - N));
        // (the weights from the last threads: other waves than the powers')
        const int wn = (job.kind == TAB_SUFFIX) ? k : P;
        for (int a = TH - 1 - tid; a >= 0 && a <= wn; a -= TH)
            wtab[a] = pow(od.p, (double)a) * pow(1.0 - od.p, (double)(wn - a));
    }
    if (job.kind == TAB_PREFIX && od.ucount) {
        // Per-lane unranking reads binomials and group offsets at divergent
        // indices: keep them in LDS (P <= kMaxUnrank is checked on the host).
        for (int e = tid; e < P * (kMaxUnrank + 1); e += TH)
            binom[e / (kMaxUnrank + 1)][e % (kMaxUnrank + 1)] = kBinom.c[e / (kMaxUnrank + 1)][e % (kMaxUnrank + 1)];
        for (int a = tid; a <= P + 1; a += TH) goff[a] = gm(od.goff)[a];
    }
    __syncthreads();

    if (job.kind == TAB_WEIGHTS) {
        // time-varying moves: the weights sit in g (scaled by 2^wexp), one
        // group; binomial exact trees with X-only records: W_a times the
        // group's multiplier c_a
        for (int a = tid; a <= P; a += TH)
            gm(od.Wg)[a] = (tv || tri) ? (a == 0 ? ldexp(1.0, -od.wexp) : 1.0)
                       : (od.xonly || (od.ucount && !od.fp32))
                           ? wtab[a] * group_cf(od, upow, a) * od.scale
                           : wtab[a];
        return;
    }

    const int lane = tid & 63;
    const bool bound = od.bnd_pre != nullptr;

    if (job.kind == TAB_SUFFIX) {
        // FP32 binomial bound: this job's histogram of v = sign Y_s (mass,
        // smallest and largest value per bin; integer atomics, so the
        // result does not depend on their order).  Neighbouring lanes hold
        // neighbouring suffixes, whose values often share a bin: lane l
        // updates copy l mod kCopies of the bin (copies side by side, in
        // different banks), and the copies are merged at the end.
        constexpr int kCopies = TH >= 1024 ? 8 : 2;
        __shared__ unsigned long long hq[kHistBins * kCopies], hlo[kHistBins * kCopies],
            hhi[kHistBins * kCopies];
        const bool hist = od.hist != nullptr;
        if (hist) {
            for (int b = tid; b < kHistBins * kCopies; b += TH) {
                hq[b] = 0ull;
                hlo[b] = ~0ull;
                hhi[b] = 0ull;
            }
            __syncthreads();
        }
        const int copy = lane % kCopies;
        // Virtual lane v (wave vw = v / 64) takes suffixes v, v + kVirt, ...
        const bool fast = !od.persuf && !tri && !tv && k <= 16;
        const int walk = walk_of(od.payoff);
        for (int vw = tid >> 6; vw < kVirtWaves; vw += TH / 64) {
            double bs[4] = {0.0, 0.0, 0.0, 0.0};  // om rhoY, om |E|, om rhoE, om
            for (int64_t i = vw * 64 + lane; i < job.count; i += kVirt) {
                const int64_t s = job.first + i;
                int b = 0;
                double sig = 0.0, mu = -INFINITY, nu = INFINITY, e = 1.0, om = 1.0;
                if (fast) {
                    // Constant-move binomial suffixes: only the quantity
                    // the payoff uses is walked (the others keep their
                    // start values, which no payoff of this kind reads).
                    const uint32_t s32 = (uint32_t)s;
                    int lev;
                    switch (walk) {
                    case WALK_SUM: lev = walk_bits<WALK_SUM>(s32, k, N, upow, sig); break;
                    case WALK_MAX: lev = walk_bits<WALK_MAX>(s32, k, N, upow, mu); break;
                    case WALK_MIN: lev = walk_bits<WALK_MIN>(s32, k, N, upow, nu); break;
                    default: lev = 2 * __popc(s32) - k; break;
                    }
                    e = upow[lev + N];
                    b = __popc(s32);
                    om = wtab[b];
                } else {
                    int lev = 0;
                    double mt = 1.0;
                    uint32_t rem = (uint32_t)s;  // trinomial digits (s < 3^12)
                    int32_t key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    for (int j = 1; j <= k; ++j) {
                        // Exact enumeration: suffix s spells its steps (first
                        // step most significant; base 3 digits for a
                        // trinomial tree).  Shared-Sample MC: suffix s is draw
                        // s, the suffix of sample s in stratum 0xFFFFFFFF of
                        // the stratified estimator (eight steps per Philox
                        // block, step_keys8).
                        int bit, dgt;  // dgt: 0 down, 1 middle, 2 up
                        if (od.persuf) {
                            const int jj = j - 1;
                            if ((jj & 7) == 0)
                                step_keys8((uint32_t)(jj >> 3), k - jj < 8 ? k - jj : 8,
                                           (uint32_t)s, 0xFFFFFFFFu, od.stream_id,
                                           (uint32_t)od.seed, (uint32_t)(od.seed >> 32), od.thr,
                                           key);
                            int32_t x = key[0];
#pragma unroll
                            for (int i2 = 1; i2 < 8; ++i2)
                                if ((jj & 7) == i2) x = key[i2];
                            bit = x < 0 ? 1 : 0;
                            dgt = 2 * bit;
                        } else if (tri) {
                            const uint32_t pw = pw3[k - j];
                            dgt = (int)(rem / pw);
                            rem -= (uint32_t)dgt * pw;
                            bit = dgt == 2;
                            om *= dgt == 2 ? od.p : (dgt == 1 ? pm : od.pd);
                        } else {
                            bit = (int)((s >> (k - j)) & 1);
                            dgt = 2 * bit;
                        }
                        b += bit;
                        lev += dgt - 1;
                        double m;
                        if (tv) {
                            // multiplier relative to the prefix end, step P + j
                            const int t = P + j - 1;
                            mt = bit ? mt * tvu[t] : mt / tvu[t];
                            om *= bit ? tvp[t] : 1.0 - tvp[t];
                            m = mt;
                        } else {
                            m = upow[lev + N];
                        }
                        sig += m;
                        mu = fmax(mu, m);
                        nu = fmin(nu, m);
                        e = m;
                    }
                    if (!tv && !tri) om = wtab[b];
                }
                double Y, E;
                suffix_map(od.payoff, sig, mu, nu, e, Y, E);
                const double Ys = (Y - od.center) * od.inv_scale;
                gm(od.Y)[s] = Ys;
                // (the FP32 binomial form centres Y per up-count group in
                // the enumeration, from Y[s])
                if (od.fp32 && !od.xonly) gm(od.Y32)[s] = (float)Ys;
                gm(od.Om)[s] = om;
                gm(od.E)[s] = E;
                if (od.dbg_b) gm(od.dbg_b)[s] = b;
                if (hist) {
                    const double v = od.sign * Ys;
                    const int hb = hist_bin(v, od.vlo, od.hw) * kCopies + copy;
                    atomicAdd(&hq[hb], (unsigned long long)ceil(om * kHistFix));
                    atomicMin(&hlo[hb], ord_of(v));
                    atomicMax(&hhi[hb], ord_of(v));
                }
                if (bound) {
                    double rY, rE;
                    suffix_err(od.payoff, sig, mu, nu, e, k, od.eps_suf, E, rY, rE);
                    rY = (rY + kU64 * fabs(Y - od.center)) * od.inv_scale;
                    if (od.fp32) rY += kU32 * fabs(Ys) + kSub32;
                    bs[0] += om * rY;
                    bs[1] += om * fabs(E);
                    bs[2] += om * rE;
                    bs[3] += om;
                }
            }
            if (bound) vsum4_lane(bs, red, vw, lane);
        }
        if (bound) {
            __syncthreads();
            if (tid < 4) {
                double t = 0.0;
                for (int w = 0; w < kVirtWaves; ++w) t += red[tid][w];
                gm(od.bnd_suf)[4 * job.chunk + tid] = t;
            }
        }
        if (hist) {
            __syncthreads();
            const auto h = gm(od.hist + (size_t)3 * kHistBins * job.chunk);
            for (int b = tid; b < kHistBins; b += TH) {
                unsigned long long q = 0ull, lo = ~0ull, hi = 0ull;
                for (int r = 0; r < kCopies; ++r) {
                    q += hq[b * kCopies + r];
                    lo = min(lo, hlo[b * kCopies + r]);
                    hi = max(hi, hhi[b * kCopies + r]);
                }
                h[b] = q;
                h[kHistBins + b] = lo;
                h[2 * kHistBins + b] = hi;
            }
        }
        return;
    }

    // TAB_PREFIX: positions [first, first + count) of chunk job.chunk.
    // Virtual lane v (wave vw = v / 64) takes positions v, v + kVirt, ...
    const double Nd = (double)N;
    const int walk = walk_of(od.payoff);
    double emax = 0.0;  // xonly: largest FP64 error of X_z - Cg[a] (this thread)
    for (int vw = tid >> 6; vw < kVirtWaves; vw += TH / 64) {
      double ps[4] = {0.0, 0.0, 0.0, 0.0};  // W U, c rhoX, c, W rhoU
      for (int64_t i = vw * 64 + lane; i < job.count; i += kVirt) {
        const int64_t q = job.first + i;
        // Binomial tables (FP32, and FP64 exact) are in up-count order (the
        // kernels share W_a, or W_a c_a, over each run of equal up-counts);
        // the others are in natural order, z = q.
        int a = 0;
        uint64_t z;
        if (od.ucount) {
            // the group: the largest a <= P with goff[a] <= q (binary search)
            int hi = P;
            while (a < hi) {
                const int mid = (a + hi + 1) >> 1;
                if (goff[mid] <= q) a = mid; else hi = mid - 1;
            }
            z = unrank(binom, q - goff[a], P, a);
        } else {
            z = (uint64_t)q;
            a = tri ? 0 : __popcll(z);
        }
        int lev = 0;
        double A = 0.0, M = -INFINITY, m = INFINITY, Sv = od.S, Wv = 1.0;
        uint32_t rem = (uint32_t)z;  // trinomial digits (z < 3^16)
        if (!tv && !tri) {
            // constant moves: only the quantity the payoff uses is walked
            // (z < 2^P fits 32 bits); the others keep their start values
            const uint32_t z32 = (uint32_t)z;
            double g;
            switch (walk) {
            case WALK_SUM: lev = walk_prefix_sum(z32, P, N, od.S, upow, A); break;
            case WALK_MAX:
                g = -INFINITY;
                lev = walk_bits<WALK_MAX>(z32, P, N, upow, g);
                M = od.S * g;
                break;
            case WALK_MIN:
                g = INFINITY;
                lev = walk_bits<WALK_MIN>(z32, P, N, upow, g);
                m = od.S * g;
                break;
            default: lev = 2 * __popc(z32) - P; break;
            }
        }
        for (int t = 1; (tv || tri) && t <= P; ++t) {
            int dgt;  // 0 down, 1 middle (trinomial), 2 up
            if (tri) {
                const uint32_t pw = pw3[P - t];
                dgt = (int)(rem / pw);
                rem -= (uint32_t)dgt * pw;
                a += dgt == 2;
                Wv *= dgt == 2 ? od.p : (dgt == 1 ? pm : od.pd);
            } else {
                dgt = ((z >> (P - t)) & 1) ? 2 : 0;
            }
            const bool up = dgt == 2;
            lev += dgt - 1;
            double St;
            if (tv) {
                // repeated multiplication along the path, weight as a product
                Sv = up ? Sv * tvu[t - 1] : Sv / tvu[t - 1];
                Wv *= up ? tvp[t - 1] : 1.0 - tvp[t - 1];
                St = Sv;
            } else {
                St = od.S * upow[lev + N];
            }
            A += St;
            M = fmax(M, St);
            m = fmin(m, St);
        }
        const double Pz = (P == 0) ? od.S : (tv ? Sv : od.S * upow[lev + N]);
        double X, cf, U;
        prefix_map(od.payoff, Nd, od.K, A, M, m, Pz, P == 0, X, cf, U);
        const double W = (tv || tri) ? Wv : wtab[a];
        const double Xs = (X - od.center) * od.inv_scale;
        // c of the clamped term as the enumeration applies it
        double c;
        // xonly: centred on the group (the enumeration centres the suffix
        // operand on the same Cg[a]; the difference is unchanged)
        const double Xc = od.xonly ? Xs - gm(od.Cg)[a] : Xs;
        if (od.xonly) {
            gm(od.XG)[q] = (float)Xc;
            c = W * group_cf(od, upow, a) * od.scale;  // = Wg[a]
        } else if (od.ucount && !od.fp32) {
            gm(od.XC)[q] = Xs;
            c = W * group_cf(od, upow, a) * od.scale;  // = Wg[a]
        } else if (od.fp32) {
            gm(od.XG)[2 * q] = (float)Xs;
            // time-varying moves: W_z rides in g (one group, Wg[0] = 2^-wexp)
            const float g = (tv || tri) ? (float)(ldexp(W, od.wexp) * cf * od.scale)
                                        : (float)(cf * od.scale);
            gm(od.XG)[2 * q + 1] = g;
            c = (tv || tri) ? ldexp((double)g, -od.wexp) : W * (double)g;
        } else {
            c = W * cf * od.scale;
            gm(od.XC)[2 * q] = Xs;
            gm(od.XC)[2 * q + 1] = c;
        }
        ps[0] += W * U;
        if (bound) {
            double rX, rU;
            prefix_err(od.payoff, Nd, od.K, A, m, Pz, P == 0, P, od.eps_pre, X, U, rX, rU);
            rX = (rX + kU64 * fabs(X - od.center)) * od.inv_scale;
            if (od.xonly) emax = fmax(emax, rX + kU64 * fabs(Xc));
            if (od.fp32) rX += kU32 * fabs(Xc) + kSub32;
            ps[1] += c * rX;
            ps[2] += c;
            ps[3] += W * rU;
        }
        if (od.dbg_z) {
            gm(od.dbg_z)[q] = z;
            gm(od.dbg_a)[q] = a;
        }
      }
      // Fixed-order sums over the virtual wave, then over the waves.
      vsum4_lane(ps, red, vw, lane);
    }
    // the chunk's largest FP64 error of X_z - Cg[a] (a maximum: any order)
    for (int off = 32; off >= 1; off >>= 1) emax = fmax(emax, __shfl_xor(emax, off));
    __shared__ double emx[TH / 64];
    if (lane == 0) emx[tid >> 6] = emax;
    __syncthreads();
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < kVirtWaves; ++w) t += red[tid][w];
        if (tid == 0) gm(od.chunkU)[job.chunk] = t;
        else if (bound) gm(od.bnd_pre)[4 * job.chunk + tid - 1] = t;
    }
    if (bound && tid == 4) {
        double m = 0.0;
        for (int w = 0; w < TH / 64; ++w) m = fmax(m, emx[w]);
        gm(od.bnd_pre)[4 * job.chunk + 3] = m;
    }
}

}  // namespace

hipError_t launch_tables(const OptDev *d_opts, const TableJob *d_jobs,
                         int njobs, int64_t entries, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    // Large jobs (a few thousand entries each) keep 1024 threads busy;
    // many small ones (a batch of small trees) run faster as 256-thread
    // workgroups.  The results do not depend on the choice.
    if (entries / njobs >= 1024)
        hipLaunchKernelGGL(table_kernel<1024>, dim3(njobs), dim3(1024), 0, s, d_opts, d_jobs);
    else
        hipLaunchKernelGGL(table_kernel<256>, dim3(njobs), dim3(256), 0, s, d_opts, d_jobs);
    return hipGetLastError();
}

}  // namespace bt
