// Host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "bt.h"

namespace bt {

struct DeviceInfo {
    bool ready = false;
    int device = -1;
    int cus = 0;
};

// Checks that the current device is a gfx950 and records its shape.
int ensure_device(DeviceInfo **out);
int hip_err(hipError_t e);
// BT_OK, BT_EINVAL or BT_ERANGE (N > max_n).
int check_option(const bt_option *o, int max_n);
bt_tuning resolve_tuning(int N, int precision, const bt_tuning *user);

// Exact plans in caller-provided device memory.
int plan_bytes(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
               size_t *bytes);
int plan_create_in(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
                   void *mem, size_t bytes, bool owns, hipStream_t s, bt_plan **out);

// Partitioned MC with caller-provided scratch.
int mc_check(const bt_option *opt, int32_t r, int32_t Rm);
size_t mc_scratch_bytes(int32_t r, int32_t Rm, int64_t *nitems, int64_t *per_item);
int mc_enqueue(const bt_option *opt, int32_t r, int32_t Rm, uint64_t seed, uint32_t stream_id,
               int32_t precision, double *d_out, void *scratch, hipStream_t s);

}  // namespace bt
