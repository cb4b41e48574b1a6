// Caching device allocator behind every device buffer of the library.
//
// hipFree waits for all work on the device, which would stall every other
// stream each time a serving slot retires a tree.  Released blocks are
// therefore kept in per-device free lists keyed by their rounded size and
// handed out again by later allocations (the smallest that fits, a large
// one up to a quarter bigger than asked); memory goes back to the runtime
// when a new block would leave less than a reserve (2 GiB or 1 % of the
// device) free for the runtime's own allocations, when an allocation fails
// (the cache is emptied and the allocation retried) or on fmddm_trim_cache.
//
// Blocks are released when their owner lets go of them, which may be
// before the work enqueued on them has run (a buffer regrown or a
// temporary going out of scope).  The releasing thread's stream scope
// (StreamScope) names the stream of that work: the block keeps that stream
// and an event recorded on it at release, and is handed to an allocation
// on the same stream at once, to one on another stream only when the
// event has completed.  Several streams (serving slots, set-up threads)
// then never share a block while the old user's work is pending.
#include "internal.h"

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

namespace fmddm {
namespace {

struct Block {
    void *p = nullptr;
    hipStream_t st = nullptr;  // the releasing scope's stream (when `ev`)
    hipEvent_t ev = nullptr;   // recorded on `st` at release; null: idle
};

struct Cache {
    std::mutex mu;
    std::map<int, std::multimap<size_t, Block>> free;  // device -> size -> blocks
    std::map<int, size_t> held;                        // device -> bytes in free lists
    std::map<int, size_t> live;                        // device -> bytes handed out
    std::map<int, std::vector<hipEvent_t>> events;     // device -> idle events
};

Cache &cache()
{
    static Cache *c = new Cache();  // never destroyed: blocks outlive static teardown
    return *c;
}

thread_local hipStream_t tl_stream = nullptr;
thread_local bool tl_set = false;

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

// (caller holds the lock) hipFree waits for the device, so blocks with
// pending work go too
void drop_all(int dev)
{
    Cache &c = cache();
    auto &fl = c.free[dev];
    for (auto &kv : fl) {
        (void)hipFree(kv.second.p);
        if (kv.second.ev) c.events[dev].push_back(kv.second.ev);
    }
    fl.clear();
    c.held[dev] = 0;
}

// (caller holds the lock) may block b serve an allocation on this thread's
// stream now?  -1: its event cannot be queried (its stream is gone): the
// caller frees it
int usable(const Block &b)
{
    if (!b.ev) return 1;
    if (tl_set && b.st == tl_stream) return 1;
    hipError_t q = hipEventQuery(b.ev);
    if (q == hipSuccess) return 1;
    if (q == hipErrorNotReady) return 0;
    (void)hipGetLastError();  // not this thread's launch error
    return -1;
}

// FMDDM_POISON_ALLOC=1 (read once): every floating-point block handed out
// is first filled with 0xFF bytes, a NaN in every double and float lane,
// on the allocating scope's stream, so a kernel that reads memory its
// owner has not written yields NaN instead of whatever the block held.
// Integer blocks (indices, counters) are left as they are.  A debugging
// aid; skipped for a stream under graph capture.
bool poison_on()
{
    static const bool on = [] {
        const char *v = std::getenv("FMDDM_POISON_ALLOC");
        return v && v[0] == '1';
    }();
    return on;
}

void poison(void *p, size_t r)
{
    if (!poison_on()) return;
    if (tl_set) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(tl_stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
            (void)hipGetLastError();
            return;
        }
        FM_HIP(hipMemsetAsync(p, 0xFF, r, tl_stream));
    } else {
        FM_HIP(hipMemset(p, 0xFF, r));
        FM_HIP(hipDeviceSynchronize());
    }
}

}  // namespace

void *dev_alloc(size_t bytes, size_t *rounded, bool fp)
{
    int dev = 0;
    FM_HIP(hipGetDevice(&dev));
    size_t r = round_size(bytes);
    *rounded = r;
    Cache &c = cache();
    {
        // the smallest cached block that fits; large ones are taken up to a
        // quarter bigger (requests of different sizes then reuse each
        // other's blocks instead of growing the cache), and keep their size
        std::lock_guard<std::mutex> g(c.mu);
        auto &fl = c.free[dev];
        const size_t slack = r <= (size_t(2) << 20) ? 0 : r / 4;
        for (auto it = fl.lower_bound(r); it != fl.end() && it->first <= r + slack;) {
            const int u = usable(it->second);
            if (u < 0) {
                // hipFree waits for the device: nothing can still use it
                (void)hipFree(it->second.p);
                (void)hipEventDestroy(it->second.ev);
                (void)hipGetLastError();
                c.held[dev] -= it->first;
                it = fl.erase(it);
                continue;
            }
            if (u == 0) {
                ++it;
                continue;
            }
            void *p = it->second.p;
            const size_t got = it->first;
            if (it->second.ev) c.events[dev].push_back(it->second.ev);
            fl.erase(it);
            c.held[dev] -= got;
            c.live[dev] += got;
            *rounded = got;
            if (fp) poison(p, got);
            return p;
        }
    }
    // the runtime allocates memory of its own on the way (kernel scratch,
    // library workspaces) and fails a launch when it cannot: keep a reserve
    // free by returning the cached blocks first when a new block would eat
    // into it
    {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
            const size_t reserve = std::max<size_t>(size_t(2) << 30, tot / 100);
            if (fr < r + reserve) {
                std::lock_guard<std::mutex> g(c.mu);
                drop_all(dev);
            }
        } else {
            (void)hipGetLastError();
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
    {
        std::lock_guard<std::mutex> g(c.mu);
        c.live[dev] += r;
    }
    if (fp) poison(p, r);
    return p;
}

void dev_release(void *p, size_t rounded)
{
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    Block b;
    b.p = p;
    if (tl_set) {
        // the work enqueued on the scope's stream so far may still use p
        auto &pool = c.events[dev];
        hipEvent_t ev = nullptr;
        if (!pool.empty()) {
            ev = pool.back();
            pool.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
        }
        if (ev && hipEventRecord(ev, tl_stream) == hipSuccess) {
            b.st = tl_stream;
            b.ev = ev;
        } else {
            // no event: wait for the stream instead
            if (ev) pool.push_back(ev);
            (void)hipGetLastError();
            (void)hipStreamSynchronize(tl_stream);
        }
    }
    c.free[dev].emplace(rounded, b);
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

void dev_stream_idle(hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    for (auto &kv : c.free[dev])
        if (kv.second.ev && kv.second.st == s) {
            c.events[dev].push_back(kv.second.ev);
            kv.second.ev = nullptr;
            kv.second.st = nullptr;
        }
}

StreamScope::StreamScope(hipStream_t s) : prev_(tl_stream), prev_set_(tl_set)
{
    tl_stream = s;
    tl_set = true;
}

StreamScope::~StreamScope()
{
    tl_stream = prev_;
    tl_set = prev_set_;
}

}  // namespace fmddm

extern "C" {
int64_t fmddm_memory_in_use(void) { return (int64_t)fmddm::dev_bytes(false); }
int64_t fmddm_memory_cached(void) { return (int64_t)fmddm::dev_bytes(true); }
int64_t fmddm_trim_cache(void) { return (int64_t)fmddm::dev_cache_trim(); }
}
