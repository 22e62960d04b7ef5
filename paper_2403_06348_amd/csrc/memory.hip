// Device memory for handles and build scratch: a small caching allocator so
// that repeated builds and workspace growth of the same sizes do not pay for
// hipMalloc/hipFree (which maps/unmaps pages and synchronizes the device) on
// every call.  Blocks are cached per device by exact size.  A block returns
// to the cache either at once (dev_free: the caller has synchronized the work
// using it) or once an event recorded on the stream of that work has
// completed (dev_free_after: nothing waits; the block is reused only after
// the event is seen complete).
#include <map>
#include <mutex>
#include <vector>

#include "alto_internal.h"
#include "memory.h"

namespace alto {

namespace {
struct Pending {
    void *p;
    hipEvent_t ev;
};

struct Cache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_blocks;
    std::map<void *, std::pair<int, size_t>> live;
    std::vector<Pending> pending;   // freed behind stream work not yet seen complete
    std::vector<hipEvent_t> events; // completed events for reuse
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

// Move a live block to the free lists (lock held).
void to_cache(Cache &c, void *p) {
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free_blocks[it->second].push_back(p);
    c.cached_bytes += it->second.second;
    c.live.erase(it);
}

// Blocks whose stream work has completed return to the free lists (lock
// held).  A pending event's query status is not left as the runtime's last
// error.
void reap(Cache &c) {
    size_t k = 0;
    for (size_t i = 0; i < c.pending.size(); i++) {
        const hipError_t q = hipEventQuery(c.pending[i].ev);
        if (q == hipSuccess) {
            to_cache(c, c.pending[i].p);
            c.events.push_back(c.pending[i].ev);
        } else {
            (void)hipGetLastError();
            c.pending[k++] = c.pending[i];
        }
    }
    c.pending.resize(k);
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
        if (!c.pending.empty()) reap(c);
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
    to_cache(c, p);
}

void dev_free_after(void *p, hipStream_t s) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.live.find(p) == c.live.end()) return;
    hipEvent_t ev = nullptr;
    if (!c.events.empty()) {
        ev = c.events.back();
        c.events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        ev = nullptr;
    }
    if (ev && hipEventRecord(ev, s) == hipSuccess) {
        c.pending.push_back({p, ev});
        return;
    }
    // no event: wait for the stream instead
    (void)hipGetLastError();
    if (ev) c.events.push_back(ev);
    (void)hipStreamSynchronize(s);
    (void)hipGetLastError();
    to_cache(c, p);
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
    if (!c.pending.empty()) reap(c);
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
