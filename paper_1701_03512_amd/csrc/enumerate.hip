// Exact enumeration of every Bernoulli path (eq. (f13)) and the
// deterministic reduction of its partial sums (eqs. (f14), (f15)).
//
// Section 3 gives each of M processes the 2^(N-r) paths behind one r-step
// prefix and sums the local values with one reduce.  Here the unit of work
// is a work item: a rectangle of `chunk` prefixes (a contiguous range of the
// up-count-ordered prefix table) times one tile of kTile = 64 * kJ suffixes.
// A wavefront takes items from a global counter (largest options first, the
// dynamic form of the paper's cyclic assignment of many partitions to few
// processes) until none is left.  Per item:
//   - each lane keeps kJ suffix operands Y_s in VGPRs for the whole item;
//   - the wave walks the prefixes; X_z and c_z are wave-uniform, so they come
//     through the scalar cache four prefixes per load and sit in SGPRs;
//   - each path costs one subtraction whose clamp modifier performs the
//     max(., 0) and one fused multiply-add into the lane's accumulator;
//   - the lane sum is weighted by the suffix weights omega_s, the wave sum
//     goes to partial[item] (FP64).  No atomics on data: the reduction kernel
//     sums each option's partials in a fixed order, so the result does not
//     depend on which wave ran which item.
//
// FP32 form: X, Y and g = c / W are FP32; prefixes are visited in up-count
// order, so every run of prefixes with the same up-count a shares the path
// weight factor W_a.  Within such a group the lane accumulates plain FP32
// runs of kKahanRun prefixes, folds each run into a Kahan (sum,
// compensation) pair, and at the group's end adds W_a * (sum - comp) to an
// FP64 accumulator.  Weights, the affine part and all reductions stay FP64.
#include "bt_internal.hpp"

namespace bt {
namespace {


typedef const __attribute__((address_space(4))) double *cdptr;
typedef const __attribute__((address_space(4))) float *cfptr;
typedef const __attribute__((address_space(4))) int64_t *ciptr;
typedef const __attribute__((address_space(4))) OptDev *coptr;

template <int SIGN>
__device__ __forceinline__ double cdiff(double y, double x)
{
    const double d = SIGN > 0 ? (y - x) : (x - y);
    return __builtin_fmin(__builtin_fmax(d, 0.0), 1.0);
}

template <int SIGN>
__device__ __forceinline__ float cdiff(float y, float x)
{
    const float d = SIGN > 0 ? (y - x) : (x - y);
    return __builtin_fminf(__builtin_fmaxf(d, 0.0f), 1.0f);
}

template <int SIGN>
__device__ __forceinline__ void prefixes_f64(cdptr xc, int64_t z0, int64_t z1,
                                             const double (&y)[kJ],
                                             double (&acc)[kJ])
{
    int64_t z = z0;
    for (; z + 4 <= z1; z += 4) {
        const double x0 = xc[2 * z + 0], c0 = xc[2 * z + 1];
        const double x1 = xc[2 * z + 2], c1 = xc[2 * z + 3];
        const double x2 = xc[2 * z + 4], c2 = xc[2 * z + 5];
        const double x3 = xc[2 * z + 6], c3 = xc[2 * z + 7];
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            double a = acc[j];
            a = __builtin_fma(c0, cdiff<SIGN>(y[j], x0), a);
            a = __builtin_fma(c1, cdiff<SIGN>(y[j], x1), a);
            a = __builtin_fma(c2, cdiff<SIGN>(y[j], x2), a);
            a = __builtin_fma(c3, cdiff<SIGN>(y[j], x3), a);
            acc[j] = a;
        }
    }
    for (; z < z1; ++z) {
        const double x0 = xc[2 * z], c0 = xc[2 * z + 1];
#pragma unroll
        for (int j = 0; j < kJ; ++j)
            acc[j] = __builtin_fma(c0, cdiff<SIGN>(y[j], x0), acc[j]);
    }
}

template <int SIGN>
__device__ __forceinline__ void prefixes_f32(cfptr xg, ciptr goff, cdptr Wg,
                                             int P, int64_t z0, int64_t z1,
                                             const float (&y)[kJ],
                                             double (&acc)[kJ])
{
    int a = 0;
    while (a < P && goff[a + 1] <= z0) ++a;
    int64_t z = z0;
    while (z < z1) {
        const int64_t gend = goff[a + 1] < z1 ? goff[a + 1] : z1;
        float ks[kJ], kc[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) ks[j] = kc[j] = 0.0f;
        while (z < gend) {
            const int64_t rend = (z + kKahanRun < gend) ? z + kKahanRun : gend;
            float run[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) run[j] = 0.0f;
            for (; z + 4 <= rend; z += 4) {
                const float x0 = xg[2 * z + 0], g0 = xg[2 * z + 1];
                const float x1 = xg[2 * z + 2], g1 = xg[2 * z + 3];
                const float x2 = xg[2 * z + 4], g2 = xg[2 * z + 5];
                const float x3 = xg[2 * z + 6], g3 = xg[2 * z + 7];
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    float r = run[j];
                    r = __builtin_fmaf(g0, cdiff<SIGN>(y[j], x0), r);
                    r = __builtin_fmaf(g1, cdiff<SIGN>(y[j], x1), r);
                    r = __builtin_fmaf(g2, cdiff<SIGN>(y[j], x2), r);
                    r = __builtin_fmaf(g3, cdiff<SIGN>(y[j], x3), r);
                    run[j] = r;
                }
            }
            for (; z < rend; ++z) {
                const float x0 = xg[2 * z], g0 = xg[2 * z + 1];
#pragma unroll
                for (int j = 0; j < kJ; ++j)
                    run[j] = __builtin_fmaf(g0, cdiff<SIGN>(y[j], x0), run[j]);
            }
            // Kahan fold of the run into (ks, kc); sum = ks - kc.
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const float yv = run[j] - kc[j];
                const float t = ks[j] + yv;
                kc[j] = (t - ks[j]) - yv;
                ks[j] = t;
            }
        }
        const double w = Wg[a];
#pragma unroll
        for (int j = 0; j < kJ; ++j)
            acc[j] = __builtin_fma(w, (double)ks[j] - (double)kc[j], acc[j]);
        ++a;
    }
}

// Broadcast of lane 0's value (all lanes are active where this is called);
// the result is known to be wave-uniform, so it lives in SGPRs.
__device__ __forceinline__ int64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t next_item(unsigned long long *counter,
                                             int lane)
{
    unsigned long long v = 0;
    if (lane == 0) v = atomicAdd(counter, 1ull);
    return uniform64(v);
}

template <bool F32>
__global__ __launch_bounds__(256) void enumerate_kernel(
    coptr opts, int nopts, int64_t nitems, unsigned long long *counter,
    double *__restrict__ partial)
{
    const int lane = threadIdx.x & 63;
    int64_t item = next_item(counter, lane);
    while (item < nitems) {
        const int64_t next = next_item(counter, lane);
        // Option owning this item: last one with item_begin <= item.
        int lo = 0, hi = nopts - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (opts[mid].item_begin <= item) lo = mid; else hi = mid - 1;
        }
        const auto &od = opts[lo];
        const int64_t local = item - od.item_begin;
        const int64_t c = local / od.tiles;
        const int64_t t = local - c * od.tiles;
        const int64_t z0 = c * od.chunk;
        const int64_t z1 = (z0 + od.chunk < od.npre) ? z0 + od.chunk : od.npre;
        const int64_t sbase = t * kTile + lane;

        double acc[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) acc[j] = 0.0;

        if (F32) {
            float y[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int64_t s = sbase + 64 * j;
                y[j] = (s < od.nsuf) ? od.Y32[s] : 0.0f;
            }
            if (od.sign > 0)
                prefixes_f32<1>((cfptr)od.XG, (ciptr)od.goff, (cdptr)od.Wg, od.P,
                                z0, z1, y, acc);
            else
                prefixes_f32<-1>((cfptr)od.XG, (ciptr)od.goff, (cdptr)od.Wg, od.P,
                                 z0, z1, y, acc);
        } else {
            double y[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int64_t s = sbase + 64 * j;
                y[j] = (s < od.nsuf) ? od.Y[s] : 0.0;
            }
            if (od.sign > 0)
                prefixes_f64<1>((cdptr)od.XC, z0, z1, y, acc);
            else
                prefixes_f64<-1>((cdptr)od.XC, z0, z1, y, acc);
        }

        const double cu = ((cdptr)od.chunkU)[c];
        double lt = 0.0;
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            const int64_t s = sbase + 64 * j;
            if (s < od.nsuf) lt = __builtin_fma(od.Om[s], __builtin_fma(od.E[s], cu, acc[j]), lt);
        }
        for (int off = 32; off >= 1; off >>= 1) lt += __shfl_xor(lt, off);
        if (lane == 0) partial[item] = lt;
        item = next;
    }
}

__global__ void reset_counter_kernel(unsigned long long *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// One wave per option: lane l sums partial[begin + l + 64 i] in order, then
// a fixed butterfly; lane 0's total times e^{-rT} is the option's value.
__global__ __launch_bounds__(64) void reduce_kernel(
    const OptDev *__restrict__ opts, const double *__restrict__ partial,
    double *__restrict__ values)
{
    const OptDev &od = opts[blockIdx.x];
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int64_t i = lane; i < od.nitems; i += 64) s += partial[od.item_begin + i];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) values[od.out_index] = od.disc * s;
}

}  // namespace

hipError_t launch_reset_counter(unsigned long long *d_counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, d_counter);
    return hipGetLastError();
}

hipError_t launch_enumerate(const OptDev *d_opts, int nopts, int64_t nitems,
                            unsigned long long *d_counter, double *d_partial,
                            int fp32, int grid, int waves, hipStream_t s)
{
    if (nopts <= 0 || nitems <= 0) return hipSuccess;
    if (waves < 1 || waves > 4) waves = 4;
    dim3 block(64 * waves);
    if (fp32)
        hipLaunchKernelGGL(enumerate_kernel<true>, dim3(grid), block, 0, s,
                           (coptr)d_opts, nopts, nitems, d_counter, d_partial);
    else
        hipLaunchKernelGGL(enumerate_kernel<false>, dim3(grid), block, 0, s,
                           (coptr)d_opts, nopts, nitems, d_counter, d_partial);
    return hipGetLastError();
}

int enumerate_max_blocks_per_cu(int fp32, int waves)
{
    int nb = 0;
    hipError_t e;
    if (fp32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(enumerate_kernel<true>), 64 * waves, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(enumerate_kernel<false>), 64 * waves, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_reduce(const OptDev *d_opts, int nopts,
                         const double *d_partial, double *d_values,
                         hipStream_t s)
{
    if (nopts <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(nopts), dim3(64), 0, s, d_opts,
                       d_partial, d_values);
    return hipGetLastError();
}

}  // namespace bt
