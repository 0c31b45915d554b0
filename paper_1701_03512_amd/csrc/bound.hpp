// Input-rounding part of the error bound of the FP32 binomial form, over
// the paths that can reach the money.
//
// The FP32 form subtracts the stored operands y_{s,a} = fl32(Y_s - Cg[a])
// and x_z = fl32(X_z - Cg[a]) (up-count group a, both scaled by 2^-e), so
// each carries a rounding error rho.  Since max(., 0) is 1-Lipschitz and
// flat below zero, path (z, s) moves the value by at most c_z om_s
// (rhoX_z + rhoY_s), and not at all when its computed difference is at
// most -(rhoX_z + rhoY_s) (then the exact difference is not positive
// either).  Summing over every path, as the table kernel's sums do, makes
// the bound of a deep out-of-the-money option many times its value; this
// kernel keeps only the paths that pass that test, so the bound of an
// option that no path can reach is exactly zero.
//
// The table kernel's suffix jobs binned the values v = sign Y_s by the
// monotone map hist_bin (bins' value sets are ordered), keeping per bin the
// mass sum om_s (fixed point, rounded up) and the exact smallest and
// largest v.  One workgroup per prefix chunk merges the suffix jobs' bins,
// forms suffix sums from the top bin down of mass, mass times largest value
// and mass times smallest value, and takes the chunk's prefixes: a prefix's
// threshold T (no suffix with v <= T can reach the money; margins for both
// roundings and for forming T) falls in bin hist_bin(T): bins below it hold
// only values below T, bins above it only values above T.  The prefix adds
// c_a (rhoX_z M + R) over the bins from the first one with a value above T,
// where M is their mass and R bounds their sum of om_s rhoY_s through the
// suffix sums: |v - C| is at most bmax - C in bins above the group's centre
// C, C - bmin in bins below it and bmax - min(bmin, C) in the bin that
// reaches past it.  Whole bins count, so the sum bounds the sum over the
// active paths from above.  Every sum runs in a fixed order; the chunk's
// total goes to bnd_pre[4c], which the reduction adds up.
//
// The workgroups run inside the FP32 binomial enumeration launch, after its
// rectangles (they need only the tables), so that they fill the launch's
// tail instead of adding a launch of their own.
#pragma once

#include "bt_internal.hpp"

namespace bt {
namespace bound {

constexpr int kBT = kHistBins;  // threads per workgroup: thread b owns bin b
static_assert(kBT == 64 * kWaves, "the enumeration's workgroups run it");
constexpr double kU64 = 0x1p-53;
constexpr double kU32 = 0x1p-24;
constexpr double kSub32 = 0x1p-149;  // FP32 rounding below the normal range
constexpr int kMaxGroups = kExactMaxN + 1;
static_assert(kMaxChunk % kBT == 0, "a chunk's operands spread evenly over the threads");

// Fixed-order block reductions (lane butterfly, then the waves in order).
__device__ inline double block_sum(double v, double *red)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kBT / 64; ++w) t += red[w];
    return t;
}
__device__ inline double block_max(double v, double *red)
{
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = red[0];
    for (int w = 1; w < kBT / 64; ++w) t = fmax(t, red[w]);
    return t;
}

// Suffix sums out_i[b] = sum_{b' >= b} v_i over the threads b' >= b (one
// entry per thread) of three values at once, out_i[kHistBins] = 0: a scan
// inside each wave from its top lane, then the totals of the waves above.
// Fixed order.
__device__ inline void suffix_scan3(double v0, double v1, double v2, double *o0, double *o1,
                             double *o2, double (*red)[kBT / 64])
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const double a0 = __shfl_down(v0, off), a1 = __shfl_down(v1, off),
                     a2 = __shfl_down(v2, off);
        if (lane + off < 64) {
            v0 += a0;
            v1 += a1;
            v2 += a2;
        }
    }
    __syncthreads();
    if (lane == 0) {  // the wave's totals
        red[0][w] = v0;
        red[1][w] = v1;
        red[2][w] = v2;
    }
    __syncthreads();
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int w2 = kBT / 64 - 1; w2 > w; --w2) {
        b0 += red[0][w2];
        b1 += red[1][w2];
        b2 += red[2][w2];
    }
    o0[tid] = v0 + b0;
    o1[tid] = v1 + b1;
    o2[tid] = v2 + b2;
    if (tid == 0) o0[kHistBins] = o1[kHistBins] = o2[kHistBins] = 0.0;
    __syncthreads();
}

// Bound sums of prefix chunk gc of the plan (all kBT threads of the
// workgroup call it).
template <typename OPTS>
__device__ void chunk(OPTS opts, int nopts, int64_t gc)
{
    int lo_o = 0, hi_o = nopts - 1;
    while (lo_o < hi_o) {
        const int mid = (lo_o + hi_o + 1) >> 1;
        if (opts[mid].chunk_begin <= gc) lo_o = mid; else hi_o = mid - 1;
    }
    const auto &od = opts[lo_o];
    const int64_t c = gc - od.chunk_begin;
    if (!od.hist || c >= od.nchunks) return;

    __shared__ double bm[kHistBins], bl[kHistBins], bh[kHistBins];
    __shared__ double Mc[kHistBins + 1], Hc[kHistBins + 1], Lc[kHistBins + 1];
    __shared__ double gC[kMaxGroups], gry[kMaxGroups], gW[kMaxGroups];
    __shared__ int gbc[kMaxGroups];
    __shared__ int64_t goff[kMaxGroups + 1];
    __shared__ double red[kBT / 64], red3[3][kBT / 64];
    __shared__ float xs[kMaxChunk];
    const int tid = threadIdx.x;
    const double sg = (double)od.sign;
    const int64_t z0 = c * od.chunk;
    const int n = (int)((z0 + od.chunk < od.npre) ? od.chunk : od.npre - z0);

    // 1. bin tid over the suffix jobs (mass, rounded up; smallest and
    // largest value) and the chunk's prefix operands: the loads of a round
    // (16 jobs, the whole chunk) are all issued before any is used, since
    // the histograms were written on other XCDs and come from memory
    unsigned long long q = 0ull, lo = ~0ull, hi = 0ull;
    constexpr int kJobsPerRound = 4;
    constexpr int kXPerThread = kMaxChunk / kBT;
    for (int j0 = 0; j0 < od.nsufjobs; j0 += kJobsPerRound) {
        unsigned long long hq[kJobsPerRound], hl[kJobsPerRound], hh[kJobsPerRound];
        float xv[kXPerThread];
#pragma unroll
        for (int i = 0; i < kJobsPerRound; ++i) {
            const bool ok = j0 + i < od.nsufjobs;
            const uint64_t *h = od.hist + (size_t)3 * kHistBins * (ok ? j0 + i : 0);
            hq[i] = ok ? h[tid] : 0ull;
            hl[i] = ok ? h[kHistBins + tid] : ~0ull;
            hh[i] = ok ? h[2 * kHistBins + tid] : 0ull;
        }
        if (j0 == 0) {
#pragma unroll
            for (int i = 0; i < kXPerThread; ++i) {
                const int zz = tid + kBT * i;
                xv[i] = zz < n ? od.XG[z0 + zz] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < kXPerThread; ++i)
                if (tid + kBT * i < n) xs[tid + kBT * i] = xv[i];
        }
#pragma unroll
        for (int i = 0; i < kJobsPerRound; ++i) {
            q += hq[i];
            lo = min(lo, hl[i]);
            hi = max(hi, hh[i]);
        }
    }
    const bool full = hi != 0ull;
    const double m = full ? __ull2double_ru(q) * (1.0 / kHistFix) : 0.0;
    const double bmin = full ? of_ord(lo) : 0.0;
    const double bmax = full ? of_ord(hi) : -INFINITY;
    bm[tid] = m;
    bl[tid] = bmin;
    bh[tid] = bmax;
    for (int a = tid; a <= od.P + 1; a += kBT) goff[a] = od.goff[a];
    suffix_scan3(m, full ? m * bmax : 0.0, full ? m * bmin : 0.0, Mc, Hc, Lc, red3);
    // the extreme values and magnitudes over the bins
    const double vmax = block_max(full ? bmax : -INFINITY, red);
    const double vmin = -block_max(full ? -bmin : -INFINITY, red);
    const double vabs = fmax(fabs(vmin), fabs(vmax));

    // 2. per group: its centre C, the first bin with a value above C (the
    // only one that can hold values on both sides of it) and the largest
    // rhoY over all values (FP64 subtraction, FP32 rounding with 2 u32 of
    // slack for the second order, the stored value's own FP64 error)
    for (int a = tid; a <= od.P; a += kBT) {
        const double C = sg * od.Cg[a];
        int bc = hist_bin(C, od.vlo, od.hw);
        if (!(bh[bc] > C)) ++bc;  // bins from bc + 1 on hold only values above C
        gC[a] = C;
        gbc[a] = bc;
        gW[a] = od.Wg[a];
        const double d = fmax(fabs(vmin - C), fabs(vmax - C));
        gry[a] = ((kU32 + kU64) * d + kSub32) * (1.0 + 2.0 * kU32) + od.eY;
    }
    __syncthreads();

    // 3. the chunk's prefixes
    const double fy = (kU32 + kU64) * (1.0 + 2.0 * kU32);
    const double cy = kSub32 * (1.0 + 2.0 * kU32) + od.eY;
    const double ex = od.bnd_pre[4 * c + 3];  // FP64 error of X_z - Cg[a] over the chunk
    double tot = 0.0;
    int a = 0;
    for (int i = tid; i < n; i += kBT) {
        const int64_t z = z0 + i;
        while (goff[a + 1] <= z) ++a;
        const double C = gC[a], rymax = gry[a];
        const double x = sg * (double)xs[i];
        const double rx = (kU32 * fabs(x) + kSub32) * (1.0 + 2.0 * kU32) + ex;
        // no suffix with v <= T can reach the money: its computed
        // difference is at most v - C + rhoY - x <= -(rhoX + rhoY)
        double T = x + C - rx - 2.0 * rymax;
        T -= 4.0 * kU64 * (fabs(x) + fabs(C) + rx + 2.0 * rymax);
        const int g = hist_bin(T, od.vlo, od.hw);
        const int b = bh[g] > T ? g : g + 1;  // bins from b on: values above T
        if (b >= kHistBins) continue;
        // sum of m |v - C| over bins b.. (see the header)
        const int bc = gbc[a];
        double D;
        if (b > bc) {
            D = Hc[b] - C * Mc[b];
        } else {
            D = C * (Mc[b] - Mc[bc]) - (Lc[b] - Lc[bc]);
            if (bc < kHistBins) {
                D += Hc[bc + 1] - C * Mc[bc + 1];
                if (bm[bc] > 0.0) D += bm[bc] * (bh[bc] - fmin(bl[bc], C));
            }
        }
        // the rounding of the suffix sums and of D's own terms
        D += 64.0 * kU64 * Mc[b] * (vabs + fabs(C));
        tot += gW[a] * ((rx + cy) * Mc[b] + fy * fmax(D, 0.0));
    }
    const double t = block_sum(tot, red);
    if (tid == 0) od.bnd_pre[4 * c] = t;
}

}  // namespace bound
}  // namespace bt
