// Device memory of plans and of the dimension-incremental driver: a per-device cache of
// released blocks.  A loop that creates and destroys plans (the driver makes one per step)
// then reuses the blocks of the previous plans instead of paying hipMalloc and hipFree
// (which waits for the whole device) every time.
//
// Blocks are allocated in size classes of four per octave (at most 25% over the request);
// a request takes the smallest cached block of its class or up to twice its class (buffers
// that grow from call to call, like the driver's candidate lists, then find the previous
// call's blocks).  A block goes back to the cache only once the device is done with it:
// every caller synchronises the stream its work ran on before dev_free.  The cache keeps
// at most an eighth of the device's memory; beyond that, and on mr1l_release_cache, blocks
// are freed.  An allocation that fails empties the device's cache and tries once more.
#include <map>
#include <mutex>
#include <unordered_map>

#include "mr1l_internal.h"

namespace mr1l {

namespace {

constexpr int kMaxDevices = 64;

struct Cache {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> free;   // class bytes -> cached blocks (none empty)
    std::unordered_map<void *, size_t> cls;       // every live or cached block
    size_t cached = 0;
    size_t limit = 0;                             // an eighth of the device memory
};

Cache g_cache[kMaxDevices];

size_t size_class(size_t b)
{
    if (b <= 256) return 256;
    const int k = 63 - __builtin_clzll((unsigned long long)(b - 1));   // 2^k < b <= 2^(k+1)
    const size_t base = size_t(1) << k, step = base / 4;
    return base + (b - base + step - 1) / step * step;
}

int current_device(int &dev)
{
    MR1L_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MR1L_E_ARG, "device index beyond the memory cache");
    return MR1L_OK;
}

void drain(Cache &c)   // with c.mu held
{
    for (auto &kv : c.free)
        for (void *q : kv.second) {
            c.cls.erase(q);
            (void)hipFree(q);
        }
    c.free.clear();
    c.cached = 0;
}

}  // namespace

int dev_alloc(void **ptr, size_t bytes)
{
    *ptr = nullptr;
    int dev = 0, rc = current_device(dev);
    if (rc) return rc;
    Cache &c = g_cache[dev];
    const size_t k = size_class(std::max<size_t>(bytes, 16));
    std::lock_guard<std::mutex> g(c.mu);
    if (c.limit == 0) {
        size_t fr = 0, total = 0;
        c.limit = hipMemGetInfo(&fr, &total) == hipSuccess && total > 0 ? total / 8 : size_t(8) << 30;
    }
    auto it = c.free.lower_bound(k);
    if (it != c.free.end() && it->first <= 2 * k) {
        *ptr = it->second.back();
        it->second.pop_back();
        c.cached -= it->first;
        if (it->second.empty()) c.free.erase(it);
        return MR1L_OK;
    }
    hipError_t e = hipMalloc(ptr, k);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        drain(c);
        e = hipMalloc(ptr, k);
    }
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(MR1L_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    c.cls[*ptr] = k;
    return MR1L_OK;
}

void dev_free(void *ptr)
{
    if (!ptr) return;
    int dev = 0;
    if (current_device(dev)) {
        (void)hipFree(ptr);
        return;
    }
    Cache &c = g_cache[dev];
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.cls.find(ptr);
    if (it == c.cls.end()) {   // not from dev_alloc on this device
        (void)hipFree(ptr);
        return;
    }
    const size_t k = it->second;
    if (c.cached + k > c.limit) {
        c.cls.erase(it);
        (void)hipFree(ptr);
        return;
    }
    c.free[k].push_back(ptr);
    c.cached += k;
}

}  // namespace mr1l

extern "C" int mr1l_release_cache(void)
{
    int dev = 0, rc = mr1l::current_device(dev);
    if (rc) return rc;
    mr1l::Cache &c = mr1l::g_cache[dev];
    std::lock_guard<std::mutex> g(c.mu);
    mr1l::drain(c);
    return MR1L_OK;
}
