// Exact batch pricing without any device allocation.
//
// bt_price_batch builds a plan (tables, partial sums, values) in device
// memory it allocates for the call.  bt_price_batch_noalloc runs the same
// plan, with the same kernels and launch shapes, inside one fixed array that
// the code object itself carries (`scratch`, kNoAllocBytes, 256-byte
// aligned), so a caller that must not allocate device memory can still
// price.  Each device the library runs on holds its own copy of the array
// from the first use of the library on that device until the process ends.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress when the library
// sets the device up (noalloc_attach, called by ensure_device with that
// device current) and only that address is ever handed to kernels and
// copies.  Nothing in the plan has to start at zero: the table kernel writes
// every table entry, the enumeration every partial slot, the reduction every
// value.  Calls on one device are serialized by a per-device lock for their
// whole duration (each call synchronizes its stream before returning), so
// two calls of one process never share the array at once.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "bt.h"
#include "bt_internal.hpp"
#include "host_common.hpp"

namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;  // 64 MiB per device

__device__ __align__(256) char scratch[kNoAllocBytes];

std::mutex g_noalloc_mu[bt::kMaxDevices];

}  // namespace

namespace bt {

int noalloc_attach(DeviceInfo *d)
{
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();  // leave no sticky error for the next call
        d->noalloc_ptr = nullptr;
        return BT_EDEVICE;
    }
    d->noalloc_ptr = ptr;
    return BT_OK;
}

}  // namespace bt

using namespace bt;

extern "C" int bt_price_batch_noalloc(const bt_option *opts, int32_t n, int32_t precision,
                                      const bt_tuning *tune, bt_result *outs, void *stream)
{
    if (!opts || !outs || n < 1) return BT_EINVAL;
    size_t bytes = 0;
    int rc = plan_bytes(opts, n, precision, tune, &bytes);
    if (rc) return rc;
    if (bytes > kNoAllocBytes) return BT_ENOMEM;
    DeviceInfo *dev = nullptr;
    rc = ensure_device(&dev);
    if (rc) return rc;
    if (!dev->noalloc_ptr) return BT_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_noalloc_mu[dev->device]);
    return plan_price_in(opts, n, precision, tune, outs, dev->noalloc_ptr, kNoAllocBytes, s);
}
