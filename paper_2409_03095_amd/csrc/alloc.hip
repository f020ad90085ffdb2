// Device-memory cache (gfx950 runtime support, host code).
//
// A call of the library makes a few tens of device allocations (records, scratch,
// pools, the output CSR); each hipMalloc / hipFree costs about 0.1 ms of host time
// while the GPU waits, which is ~10 % of a step of the benchmark workload. Freed
// blocks are therefore kept per device in size classes (powers of two up to
// 256 MiB, multiples of 64 MiB above) and handed out again:
//  - a block released stream-ordered on stream s (dev_release) is reused only by
//    allocations on s, which run after every earlier use of the block on s;
//  - a block released idle (dev_release_idle, after a device synchronisation) is
//    reused on any stream.
// The cache holds at most a quarter of the device's memory; releases beyond that
// go back to the driver. mcmi_cache_trim returns every cached block.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace mcmi {
namespace {

struct Cached {
    void *p;
    size_t bytes;
    hipStream_t stream;  // the stream of a stream-ordered release (the null stream too)
    bool idle;           // released after a device synchronisation: reusable on any stream
    int device;
};

struct Cache {
    std::mutex mu;
    std::unordered_map<void *, std::pair<size_t, int>> live;  // ptr -> (class bytes, device)
    std::vector<Cached> free_blocks;
    size_t cached_bytes = 0;
};

Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: the driver may be gone at exit
    return *c;
}

size_t size_class(size_t bytes) {
    if (bytes < 4096) bytes = 4096;
    const size_t big = (size_t)256 << 20;
    if (bytes <= big) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        return c;
    }
    const size_t step = (size_t)64 << 20;
    return (bytes + step - 1) / step * step;
}

size_t cache_limit(int device) {
    static size_t limit[64] = {0};
    if (device < 0 || device >= 64) return 0;
    if (!limit[device]) {
        size_t free_b = 0, total_b = 0;
        limit[device] = hipMemGetInfo(&free_b, &total_b) == hipSuccess ? total_b / 4 : ((size_t)1 << 30);
    }
    return limit[device];
}

void release(void *p, hipStream_t s, bool idle) {
    if (!p) return;
    Cache &c = cache();
    std::unique_lock<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) {  // not ours: hand it back to the driver
        lk.unlock();
        (void)hipFree(p);
        return;
    }
    const size_t bytes = it->second.first;
    const int dev = it->second.second;
    c.live.erase(it);
    if (c.cached_bytes + bytes > cache_limit(dev)) {
        lk.unlock();
        (void)hipFree(p);  // synchronises the device: every earlier use has completed
        return;
    }
    c.free_blocks.push_back({p, bytes, s, idle, dev});
    c.cached_bytes += bytes;
}

}  // namespace

hipError_t dev_alloc(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t cls = size_class(bytes);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        for (size_t i = c.free_blocks.size(); i-- > 0;) {
            Cached &b = c.free_blocks[i];
            if (b.bytes == cls && b.device == dev && (b.idle || b.stream == s)) {
                *p = b.p;
                c.cached_bytes -= b.bytes;
                c.free_blocks[i] = c.free_blocks.back();
                c.free_blocks.pop_back();
                c.live[*p] = {cls, dev};
                return hipSuccess;
            }
        }
    }
    e = hipMalloc(p, cls);
    if (e != hipSuccess) {
        // the cache may hold the memory: return it and try once more
        mcmi_cache_trim();
        (void)hipGetLastError();
        e = hipMalloc(p, cls);
        if (e != hipSuccess) {
            *p = nullptr;
            return e;
        }
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.live[*p] = {cls, dev};
    return hipSuccess;
}

void dev_release(void *p, hipStream_t s) { release(p, s, false); }

void dev_release_idle(void *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    release(p, nullptr, true);
}

}  // namespace mcmi

extern "C" void mcmi_cache_trim(void) {
    using namespace mcmi;
    Cache &c = cache();
    std::vector<Cached> blocks;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        blocks.swap(c.free_blocks);
        c.cached_bytes = 0;
    }
    if (blocks.empty()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (const Cached &b : blocks) {
        (void)hipSetDevice(b.device);
        (void)hipFree(b.p);  // synchronises that device: stream-ordered releases are complete
    }
    (void)hipSetDevice(cur);
}
