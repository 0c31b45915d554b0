// Device buffers for the synchronous one-shot calls (bt_price_exact,
// bt_price_batch, their time-varying and trinomial forms, bt_price_stratified,
// bt_price_mc).  Each such call builds its plan or Monte Carlo scratch in a
// buffer taken from a per-device cache and gives it back after its last
// synchronisation, so after the first calls of a given size no call
// allocates or frees device memory (hipFree would also synchronise the whole
// device).  Buffers are sized up to a power of two of at least 1 MiB; a
// buffer is never shared by two calls at once (calls on different threads
// and streams take different buffers).  Idle buffers above kMaxIdleBytes in
// total are freed when a new one has to be allocated; the rest stay with the
// process until it ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "bt.h"
#include "bt_internal.hpp"
#include "host_common.hpp"

namespace bt {
namespace {

constexpr size_t kMinBlock = (size_t)1 << 20;
constexpr size_t kMaxIdleBytes = (size_t)2 << 30;

struct Block {
    void *ptr;
    size_t size;
    bool busy;
};

struct DevicePool {
    std::mutex mu;
    std::vector<Block> blocks;
};

DevicePool g_pool[kMaxDevices];

size_t block_size(size_t bytes)
{
    size_t s = kMinBlock;
    while (s < bytes) s <<= 1;
    return s;
}

}  // namespace

int pool_acquire(size_t bytes, void **ptr, size_t *cap)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BT_EDEVICE;
    DevicePool &P = g_pool[dev];
    std::lock_guard<std::mutex> lk(P.mu);
    Block *best = nullptr;
    for (Block &b : P.blocks)
        if (!b.busy && b.size >= bytes && (!best || b.size < best->size)) best = &b;
    if (best) {
        best->busy = true;
        *ptr = best->ptr;
        *cap = best->size;
        return BT_OK;
    }
    // Free idle buffers beyond the cache's limit (largest first) before
    // allocating another.
    const size_t want = block_size(bytes);
    size_t idle = 0;
    for (const Block &b : P.blocks)
        if (!b.busy) idle += b.size;
    std::sort(P.blocks.begin(), P.blocks.end(),
              [](const Block &a, const Block &b) { return a.size > b.size; });
    for (auto it = P.blocks.begin(); it != P.blocks.end() && idle + want > kMaxIdleBytes;) {
        if (!it->busy) {
            idle -= it->size;
            (void)hipFree(it->ptr);
            it = P.blocks.erase(it);
        } else {
            ++it;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return BT_ENOMEM;
    }
    P.blocks.push_back(Block{p, want, true});
    *ptr = p;
    *cap = want;
    return BT_OK;
}

void pool_release(void *ptr)
{
    int dev = -1;
    if (!ptr || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    DevicePool &P = g_pool[dev];
    std::lock_guard<std::mutex> lk(P.mu);
    for (Block &b : P.blocks)
        if (b.ptr == ptr) {
            b.busy = false;
            return;
        }
}

}  // namespace bt
