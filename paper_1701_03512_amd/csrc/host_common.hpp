// Host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "bt.h"

namespace bt {

constexpr int kMaxDevices = 64;

struct DeviceInfo {
    bool ready = false;
    int device = -1;
    int cus = 0;
    void *noalloc_ptr = nullptr;  // device address of the fixed no-allocation array
};

// Checks that the current device is a gfx950 and records its shape; the
// first call on a device also looks up that device's address of the
// no-allocation array (noalloc_attach).
int ensure_device(DeviceInfo **out);
// hipGetSymbolAddress of the no-allocation array on the current device into
// d->noalloc_ptr (nullptr and BT_EDEVICE if the lookup fails).
int noalloc_attach(DeviceInfo *d);
int hip_err(hipError_t e);
// BT_OK, BT_EINVAL or BT_ERANGE (N > max_n).
int check_option(const bt_option *o, int max_n);
// Launch shape for depth N: the built-in rule and then the autotuned table
// (or `depth_table`[N] in its place, when given), or (one_tree) the shape
// for one tree at a time; then the caller's non-zero fields.
bt_tuning resolve_tuning(int N, int precision, const bt_tuning *user, bool one_tree = false,
                         const bt_tuning *depth_table = nullptr);

// Extra shape of a one-option plan.
//  shared: Shared-Sample Monte Carlo (Section 4, Remark): the first r steps
//          enumerated, R drawn suffixes of N - r steps;
//  tv_u, tv_p: time-varying moves (the case after eq. (f12)), host arrays of
//          N entries, step t at index t - 1 (nullptr: the option's u and p);
//  tri:    a trinomial tree (3^N paths): up u with probability opt.p, middle
//          1 with 1 - opt.p - pd, down 1/u with pd.
struct PlanSpec {
    bool tri = false;
    double pd = 0.0;
    bool shared = false;
    int r = 0;
    int64_t R = 0;
    uint64_t seed = 0;
    uint32_t stream_id = 0;
    const double *tv_u = nullptr;
    const double *tv_p = nullptr;
    bool one_tree_shape = false;  // shapes for one tree at a time (the server)
    // per-depth shapes in place of the autotuned table (kExactMaxN + 1
    // entries, zero fields: built-in), for timing a candidate rule
    const bt_tuning *depth_table = nullptr;
};

// Plans in caller-provided device memory (ps: extra shape, or nullptr).
int plan_bytes(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
               size_t *bytes, const PlanSpec *ps = nullptr);
int plan_create_in(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
                   void *mem, size_t bytes, bool owns, hipStream_t s, bt_plan **out,
                   const PlanSpec *ps = nullptr);
int plan_shared_combine(bt_plan *pl, double *d_out3, hipStream_t s);
// One synchronous pricing pass in device memory `mem` of `bytes` (>=
// plan_bytes): the plan's uploads, tables, enumeration, reduction and the
// results into outs, all on s, with one synchronisation at the end (also
// when a step fails, so that nothing uses mem after the return).
int plan_price_in(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
                  bt_result *outs, void *mem, size_t bytes, hipStream_t s,
                  const PlanSpec *ps = nullptr);

// Device buffers of the synchronous one-shot calls (per-device cache):
// a buffer of at least `bytes` (its size in *cap) for the calling thread
// alone until pool_release.
int pool_acquire(size_t bytes, void **ptr, size_t *cap);
void pool_release(void *ptr);

// Partitioned MC with caller-provided scratch.
int mc_check(const bt_option *opt, int32_t r, int32_t Rm);
size_t mc_scratch_bytes(int32_t r, int32_t Rm, int64_t *nitems, int64_t *per_item);
// R_total > 0: proportional allocation R_m = max(1, round(R_total P(D_m)))
// (Rm is then ignored); 0: R_m = Rm in every stratum.
int mc_enqueue(const bt_option *opt, int32_t r, int32_t Rm, uint64_t seed, uint32_t stream_id,
               int32_t precision, double *d_out, void *scratch, hipStream_t s,
               uint64_t R_total = 0);

}  // namespace bt
