// Device memory for handles and build scratch: a small caching allocator so
// that repeated builds and workspace growth of the same sizes do not pay for
// hipMalloc/hipFree (which maps/unmaps pages and synchronizes the device) on
// every call.  Blocks are cached per device by exact size.  A block is only
// returned to the cache by code that has synchronized the work using it.
#include <map>
#include <mutex>
#include <vector>

#include "alto_internal.h"
#include "memory.h"

namespace alto {

namespace {
struct Cache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_blocks;
    std::map<void *, std::pair<int, size_t>> live;
    size_t cached_bytes = 0;
};

Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: avoids teardown order issues with the HIP runtime
    return *c;
}

size_t round_size(size_t b) {
    const size_t g = size_t(1) << 21;  // 2 MiB granules
    return (b + g - 1) / g * g;
}
}  // namespace

hipError_t dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t sz = round_size(bytes);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.free_blocks.find({dev, sz});
        if (it != c.free_blocks.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            c.cached_bytes -= sz;
            c.live[*p] = {dev, sz};
            return hipSuccess;
        }
    }
    e = hipMalloc(p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give the cache back to the device and retry once
        release_cached();
        e = hipMalloc(p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return e;
        }
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.live[*p] = {dev, sz};
    return hipSuccess;
}

void dev_free(void *p) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free_blocks[it->second].push_back(p);
    c.cached_bytes += it->second.second;
    c.live.erase(it);
}

size_t dev_size(void *p) {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    return it == c.live.end() ? 0 : it->second.second;
}

void release_cached() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : c.free_blocks) {
        if (kv.second.empty()) continue;
        (void)hipSetDevice(kv.first.first);
        for (void *p : kv.second) (void)hipFree(p);
        c.cached_bytes -= kv.first.second * kv.second.size();
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

size_t cached_bytes() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    return c.cached_bytes;
}

}  // namespace alto
