// Host side of the Partitioned Monte Carlo estimator (Section 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "bt.h"
#include "bt_internal.hpp"
#include "host_common.hpp"

using namespace bt;

namespace bt {

// Threshold of the integer Bernoulli draw: up iff word < floor(p 2^32).
static uint32_t up_threshold(double p)
{
    const double t = std::floor(std::ldexp(p, 32));
    if (t >= 4294967296.0) return 0xFFFFFFFFu;
    return t <= 0 ? 0u : (uint32_t)t;
}

int mc_check(const bt_option *opt, int32_t r, int32_t Rm)
{
    int rc = check_option(opt, kMcMaxN);
    if (rc) return rc;
    if (r < 0 || r >= opt->N || r > 30 || Rm < 1) return BT_EINVAL;
    if ((double)Rm * std::ldexp(1.0, r) > std::ldexp(1.0, 40)) return BT_ERANGE;
    return BT_OK;
}

// Scratch bytes for one estimate: partials (4 doubles per work item) +
// counter.
size_t mc_scratch_bytes(int32_t r, int32_t Rm, int64_t *nitems_out, int64_t *per_item_out)
{
    int64_t per_item, nitems;
    if (r == 0) {
        per_item = 4096;  // samples per item
        nitems = ((int64_t)Rm + per_item - 1) / per_item;
    } else {
        // strata per work item: 64, or more when R_m < 64, so that an item
        // holds about 4096 paths and the work counter is not the bottleneck.
        // Smaller estimates instead shrink the items so that more waves share
        // the work: down to 1024 paths each until there are 2048 items, and
        // an estimate of at most 2^20 paths (a serving pilot) down to 256
        // paths until there are 16384, so that it spreads over every SIMD
        // (2^18 paths: 53 us instead of 69).  Larger estimates keep the
        // coarser items: on a server they share the device with other
        // requests, and occupying all of it cost the concurrent exact
        // requests 40% of their median latency.
        per_item = 64;
        while (per_item < 4096 && per_item * (int64_t)Rm < 4096) per_item <<= 1;
        const int64_t ns = (int64_t)1 << r;
        const bool small = ns * (int64_t)Rm <= ((int64_t)1 << 20);
        const int64_t want_items = small ? 16384 : 2048, floor_paths = small ? 256 : 1024;
        while (per_item > 1 && (ns + per_item - 1) / per_item < want_items &&
               (per_item >> 1) * (int64_t)Rm >= floor_paths)
            per_item >>= 1;
        nitems = (ns + per_item - 1) / per_item;
    }
    if (nitems_out) *nitems_out = nitems;
    if (per_item_out) *per_item_out = per_item;
    return (size_t)nitems * 32 + 256;
}

// Enqueue the estimate with caller-provided scratch (>= mc_scratch_bytes).
// R_m = max(1, round(R P(D_m))) for a stratum with a ups among r steps;
// P(D_m) computed as the oracle does, p^a (1-p)^(r-a).
static uint32_t proportional_rm(uint64_t R, double p, int r, int a)
{
    const double W = std::pow(p, a) * std::pow(1.0 - p, r - a);
    double x = std::floor((double)R * W + 0.5);
    if (x < 1.0) x = 1.0;
    if (x > 4294967295.0) x = 4294967295.0;
    return (uint32_t)x;
}

uint64_t proportional_paths(uint64_t R, double p, int r)
{
    uint64_t tot = 0, c = 1;  // C(r, a)
    for (int a = 0; a <= r; ++a) {
        tot += c * proportional_rm(R, p, r, a);
        c = c * (uint64_t)(r - a) / (uint64_t)(a + 1);
    }
    return tot;
}

int mc_enqueue(const bt_option *opt, int32_t r, int32_t Rm, uint64_t seed,
               uint32_t stream_id, int32_t precision, double *d_out, void *scratch,
               hipStream_t s, uint64_t R_total)
{
    DeviceInfo *dev = nullptr;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    int64_t nitems = 0, per_item = 0;
    mc_scratch_bytes(r, Rm, &nitems, &per_item);
    McArgs a;
    std::memset(&a, 0, sizeof(a));
    a.S = opt->S; a.u = opt->u; a.p = opt->p; a.K = opt->K;
    a.disc = std::exp(-opt->r * opt->T);
    a.N = opt->N; a.N_d = (double)opt->N; a.r = r; a.L = opt->N - r;
    a.payoff = opt->payoff;
    a.Rm = (uint32_t)Rm;
    a.thr = up_threshold(opt->p);
    a.stream_id = stream_id;
    a.seed = seed;
    a.nstrata = (int64_t)1 << r;
    a.per_item = per_item;
    a.nitems = nitems;
    if (R_total > 0) {
        a.proportional = 1;
        for (int u = 0; u <= r; ++u) a.rm_of_a[u] = proportional_rm(R_total, opt->p, r, u);
        // at least 16 draws per stratum on average: the lane kernel, strata
        // in up-count order; fewer: the flat kernel, which packs the draws
        a.by_count = (R_total >> r) >= 16 ? 1u : 0u;
    }
    char *base = static_cast<char *>(scratch);
    unsigned long long *counter = reinterpret_cast<unsigned long long *>(base);
    double *partial = reinterpret_cast<double *>(base + 256);
    const int fp32 = precision == BT_FP32_KAHAN;
    int grid = mc_max_blocks_per_cu(fp32) * dev->cus;
    const int64_t need = (nitems + 3) / 4;
    if (grid > need) grid = (int)std::max<int64_t>(1, need);
    // At most four items per wave on average (4 waves per workgroup): take
    // them cyclically, without the atomic counter, whose serialised first
    // atomics would dominate so short a launch.  Proportional allocation
    // keeps the counter: its items differ in cost.
    const bool cyclic = !a.proportional && nitems <= (int64_t)grid * 4 * 4;
    unsigned long long *ctr = cyclic ? nullptr : counter;
    rc = cyclic ? BT_OK : hip_err(launch_reset_counter(counter, s));
    if (!rc) rc = hip_err(launch_mc(a, fp32, partial, ctr, grid, s));
    // The 1/(R_m - 1) form is NaN unless some stratum has R_m > 1.
    uint32_t rmax = a.proportional ? 0u : a.Rm;
    if (a.proportional)
        for (int u = 0; u <= r; ++u) rmax = std::max(rmax, a.rm_of_a[u]);
    const double var_scale = a.proportional ? 1.0 / ((double)R_total * (double)R_total) : 1.0;
    const double paths = a.proportional ? (double)proportional_paths(R_total, opt->p, r)
                                        : std::ldexp((double)Rm, r);
    if (!rc)
        rc = hip_err(launch_mc_combine(partial, nitems, r == 0, rmax, a.disc, var_scale, paths,
                                       d_out, s));
    return rc;
}

}  // namespace bt

extern "C" int bt_enqueue_stratified(const bt_option *opt, int32_t prefix_steps,
                                     int32_t samples_per_stratum, uint64_t seed,
                                     uint32_t stream_id, int32_t precision, double *d_out,
                                     void *stream)
{
    if (!d_out || (precision != BT_FP64 && precision != BT_FP32_KAHAN)) return BT_EINVAL;
    int rc = mc_check(opt, prefix_steps, samples_per_stratum);
    if (rc) return rc;
    rc = ensure_device(nullptr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = mc_scratch_bytes(prefix_steps, samples_per_stratum, nullptr, nullptr);
    void *scratch = nullptr;
    if (hipMallocAsync(&scratch, bytes, s) != hipSuccess) return BT_ENOMEM;
    rc = mc_enqueue(opt, prefix_steps, samples_per_stratum, seed, stream_id, precision, d_out,
                    scratch, s);
    (void)hipFreeAsync(scratch, s);
    return rc;
}

extern "C" int bt_price_stratified(const bt_option *opt, int32_t prefix_steps,
                                   int32_t samples_per_stratum, uint64_t seed,
                                   uint32_t stream_id, int32_t precision, bt_result *out,
                                   void *stream)
{
    if (!out || (precision != BT_FP64 && precision != BT_FP32_KAHAN)) return BT_EINVAL;
    int rc = mc_check(opt, prefix_steps, samples_per_stratum);
    if (rc) return rc;
    rc = ensure_device(nullptr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // [scratch | 4 outputs] in one buffer of the one-shot cache
    const size_t sb = (mc_scratch_bytes(prefix_steps, samples_per_stratum, nullptr, nullptr) +
                       255) & ~(size_t)255;
    void *mem = nullptr;
    size_t cap = 0;
    rc = pool_acquire(sb + 256, &mem, &cap);
    if (rc) return rc;
    double *d_out = reinterpret_cast<double *>(static_cast<char *>(mem) + sb);
    rc = mc_enqueue(opt, prefix_steps, samples_per_stratum, seed, stream_id, precision, d_out,
                    mem, s);
    double h[4] = {0, 0, 0, 0};
    if (!rc && hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = BT_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = BT_EDEVICE;
    pool_release(mem);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->value = h[0];
    out->var_est = h[1];
    out->var_unbiased = h[2];
    out->var_plain = h[3];
    out->std_err = std::sqrt(h[1]);
    out->err_bound = out->std_err;  // statistical: one standard error
    out->paths = (uint64_t)samples_per_stratum << prefix_steps;
    out->split = prefix_steps;
    out->status = BT_OK;
    return BT_OK;
}

extern "C" int bt_mc_debug_bits(uint64_t seed, uint32_t stream_id, uint32_t z, uint32_t m,
                                int32_t L, double p, int32_t *bits, void *stream)
{
    if (!bits || L < 1 || L > 64 || !(p > 0.0 && p < 1.0)) return BT_EINVAL;
    int rc = ensure_device(nullptr);
    if (rc) return rc;
    int32_t *d = nullptr;
    if (hipMalloc(&d, 64 * sizeof(int32_t)) != hipSuccess) return BT_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    rc = hip_err(launch_mc_bits(seed, stream_id, z, m, L, up_threshold(p), d, s));
    if (!rc && (hipMemcpyAsync(bits, d, L * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
        rc = BT_EDEVICE;
    (void)hipFree(d);
    return rc;
}

extern "C" int bt_price_mc(const bt_option *opt, int32_t estimator, int32_t prefix_steps,
                           uint64_t samples, uint64_t seed, uint32_t stream_id,
                           int32_t precision, bt_result *out, void *stream)
{
    if (!out || (precision != BT_FP64 && precision != BT_FP32_KAHAN) || samples < 1)
        return BT_EINVAL;
    // One stratum (r = 0): proportional allocation is equal allocation.
    if (estimator == BT_MC_PARTITIONED || (estimator == BT_MC_PROPORTIONAL && prefix_steps == 0)) {
        if (samples > 0x7FFFFFFFull) return BT_ERANGE;
        return bt_price_stratified(opt, prefix_steps, (int32_t)samples, seed, stream_id,
                                   precision, out, stream);
    }
    int rc = mc_check(opt, prefix_steps, 1);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    double h[4] = {0, 0, 0, NAN};  // Shared-Sample: no plain-MC variance
    uint64_t paths = 0;
    if (estimator == BT_MC_PROPORTIONAL) {
        // R_m <= R <= 2^30 keeps every per-stratum draw index and loop bound
        // far inside 32 bits.
        if (samples > ((uint64_t)1 << 30)) return BT_ERANGE;
        rc = ensure_device(nullptr);
        if (rc) return rc;
        // work items sized by the mean draws per stratum
        const int32_t rm_mean = (int32_t)std::max<uint64_t>(1, samples >> prefix_steps);
        const size_t bytes = mc_scratch_bytes(prefix_steps, rm_mean, nullptr, nullptr);
        const size_t sb = (bytes + 255) & ~(size_t)255;
        void *vmem = nullptr;
        size_t cap = 0;
        rc = pool_acquire(sb + 256, &vmem, &cap);
        if (rc) return rc;
        char *mem = static_cast<char *>(vmem);
        double *d_out = reinterpret_cast<double *>(mem + sb);
        rc = mc_enqueue(opt, prefix_steps, rm_mean, seed, stream_id, precision, d_out, mem, s,
                        samples);
        if (!rc && hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = BT_EDEVICE;
        if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = BT_EDEVICE;
        pool_release(mem);
        paths = proportional_paths(samples, opt->p, prefix_steps);
    } else if (estimator == BT_MC_SHARED_SAMPLE) {
        if (samples > ((uint64_t)1 << 31) || prefix_steps > 26) return BT_ERANGE;
        PlanSpec ss;
        ss.shared = true;
        ss.r = prefix_steps;
        ss.R = (int64_t)samples;
        ss.seed = seed;
        ss.stream_id = stream_id;
        size_t bytes = 0;
        rc = plan_bytes(opt, 1, precision, nullptr, &bytes, &ss);
        if (rc) return rc;
        rc = ensure_device(nullptr);
        if (rc) return rc;
        const size_t pb = (bytes + 255) & ~(size_t)255;
        void *vmem = nullptr;
        size_t cap = 0;
        rc = pool_acquire(pb + 256, &vmem, &cap);
        if (rc) return rc;
        char *mem = static_cast<char *>(vmem);
        double *d_out = reinterpret_cast<double *>(mem + pb);  // 3 outputs
        bt_plan *pl = nullptr;
        rc = plan_create_in(opt, 1, precision, nullptr, mem, bytes, false, s, &pl, &ss);
        if (!rc) rc = bt_plan_tables(pl, s);
        if (!rc) rc = bt_plan_enumerate(pl, s);
        if (!rc) rc = plan_shared_combine(pl, d_out, s);
        if (!rc && hipMemcpyAsync(h, d_out, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = BT_EDEVICE;
        if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = BT_EDEVICE;
        if (pl) bt_plan_destroy(pl);
        pool_release(mem);
        paths = samples << prefix_steps;
    } else {
        return BT_EINVAL;
    }
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->value = h[0];
    out->var_est = h[1];
    out->var_unbiased = h[2];
    out->var_plain = h[3];
    out->std_err = std::sqrt(h[1]);
    out->err_bound = out->std_err;  // statistical: one standard error
    out->paths = paths;
    out->split = prefix_steps;
    out->status = BT_OK;
    return BT_OK;
}
