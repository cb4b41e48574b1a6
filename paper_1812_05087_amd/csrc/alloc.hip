// Caching device allocator behind every device buffer of the library.
//
// hipFree waits for all work on the device, which would stall every other
// stream each time a serving slot retires a tree.  Released blocks are
// therefore kept in per-device free lists keyed by their rounded size and
// handed out again by later allocations; memory goes back to the runtime
// only when an allocation fails (the cache is emptied and the allocation
// retried) or on fmddm_trim_cache.  A block must not be released while
// work that uses it may still run: trees are freed only after their
// stream has drained.
#include "internal.h"

#include <map>
#include <mutex>

namespace fmddm {
namespace {

struct Cache {
    std::mutex mu;
    std::map<int, std::multimap<size_t, void *>> free;  // device -> size -> blocks
    std::map<int, size_t> held;                        // device -> bytes in free lists
    std::map<int, size_t> live;                        // device -> bytes handed out
};

Cache &cache()
{
    static Cache *c = new Cache();  // never destroyed: blocks outlive static teardown
    return *c;
}

// 512-byte granules below 2 MiB rounded to a power of two, above that to
// 2 MiB multiples
size_t round_size(size_t b)
{
    if (b <= 512) return 512;
    if (b < (size_t(2) << 20)) {
        size_t r = 512;
        while (r < b) r <<= 1;
        return r;
    }
    size_t g = size_t(2) << 20;
    return (b + g - 1) / g * g;
}

void drop_all(int dev)
{
    Cache &c = cache();
    auto &fl = c.free[dev];
    for (auto &kv : fl) (void)hipFree(kv.second);
    fl.clear();
    c.held[dev] = 0;
}

}  // namespace

void *dev_alloc(size_t bytes, size_t *rounded)
{
    int dev = 0;
    FM_HIP(hipGetDevice(&dev));
    size_t r = round_size(bytes);
    *rounded = r;
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto &fl = c.free[dev];
        auto it = fl.find(r);
        if (it != fl.end()) {
            void *p = it->second;
            fl.erase(it);
            c.held[dev] -= r;
            c.live[dev] += r;
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> g(c.mu);
            drop_all(dev);
        }
        e = hipMalloc(&p, r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error{FMDDM_ENOMEM, "device allocation of " + std::to_string(r) + " bytes failed"};
        }
    }
    FM_HIP(e);
    std::lock_guard<std::mutex> g(c.mu);
    c.live[dev] += r;
    return p;
}

void dev_release(void *p, size_t rounded)
{
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    c.free[dev].emplace(rounded, p);
    c.held[dev] += rounded;
    c.live[dev] -= rounded;
}

size_t dev_bytes(bool cached)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    return cached ? c.held[dev] : c.live[dev];
}

size_t dev_cache_trim()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    size_t h = c.held[dev];
    drop_all(dev);
    return h;
}

}  // namespace fmddm

extern "C" {
int64_t fmddm_memory_in_use(void) { return (int64_t)fmddm::dev_bytes(false); }
int64_t fmddm_memory_cached(void) { return (int64_t)fmddm::dev_bytes(true); }
int64_t fmddm_trim_cache(void) { return (int64_t)fmddm::dev_cache_trim(); }
}
