// Caching device allocator of the library.
//
// Forests and the per-call workspaces of the kNN stage are large (tens of GB at a million
// points) and are requested again and again with the same sizes.  Mapping fresh memory for
// every call costs milliseconds to seconds, so blocks obtained from hipMalloc are kept per
// device and handed out again.  A block given back records an event on the stream that
// last used it; a later request on another stream makes its own stream wait for that event
// before the block is touched, so reuse never races with work still queued.
//
// Policy: best fit among idle blocks of the device that are at most twice the request (plus
// 4 KiB); otherwise a new hipMalloc.  When hipMalloc fails, every idle block of the device
// is released and the allocation is tried once more.  rpf_release_cached_memory() returns
// all idle blocks to the runtime.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>

#include "rpf_internal.h"

namespace rpf {
namespace {

struct Block {
    void *p = nullptr;
    size_t size = 0;
    int dev = 0;
    hipStream_t last = nullptr;
    hipEvent_t ev = nullptr;
    bool pending = false;  // `ev` marks the end of the last use
};

struct Cache {
    std::mutex mu;
    std::multimap<size_t, Block *> idle[64];
    std::unordered_map<void *, Block *> live;
    uint64_t held[64] = {};
};

Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: blocks may outlive static destructors
    return *c;
}

size_t round_size(size_t b) {
    if (b == 0) b = 1;
    if (b <= ((size_t)1 << 20)) return (b + 511) & ~(size_t)511;
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

void release_idle(Cache &c, int dev) {
    for (auto &kv : c.idle[dev]) {
        Block *b = kv.second;
        if (b->ev) hipEventDestroy(b->ev);
        hipFree(b->p);
        c.held[dev] -= b->size;
        delete b;
    }
    c.idle[dev].clear();
}

}  // namespace

void *cache_alloc(size_t bytes, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    const size_t need = round_size(bytes);
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto &pool = c.idle[dev];
    auto it = pool.lower_bound(need);
    if (it != pool.end() && it->first <= 2 * need + 4096) {
        Block *b = it->second;
        pool.erase(it);
        if (b->pending && b->last != s) hipStreamWaitEvent(s, b->ev, 0);
        b->last = s;
        b->pending = false;
        c.live[b->p] = b;
        return b->p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        release_idle(c, dev);
        if (hipMalloc(&p, need) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    Block *b = new Block();
    b->p = p;
    b->size = need;
    b->dev = dev;
    b->last = s;
    c.live[p] = b;
    c.held[dev] += need;
    return p;
}

void cache_free(void *p, hipStream_t s) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    Block *b = it->second;
    c.live.erase(it);
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != b->dev) hipSetDevice(b->dev);
    if (!b->ev) hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    b->pending = b->ev && hipEventRecord(b->ev, s) == hipSuccess;
    b->last = s;
    if (cur != b->dev) hipSetDevice(cur);
    c.idle[b->dev].emplace(b->size, b);
}

void cache_free_idle(void *p) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    Block *b = it->second;
    c.live.erase(it);
    b->pending = false;  // nothing queued uses it: no event to wait for
    c.idle[b->dev].emplace(b->size, b);
}

uint64_t cache_held_bytes(int dev) {
    if (dev < 0 || dev >= 64) return 0;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    return c.held[dev];
}

void cache_release(int dev) {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    int cur = 0;
    hipGetDevice(&cur);
    for (int d = 0; d < 64; d++) {
        if ((dev >= 0 && d != dev) || c.idle[d].empty()) continue;
        hipSetDevice(d);
        release_idle(c, d);
    }
    hipSetDevice(cur);
}

}  // namespace rpf

extern "C" rpf_status rpf_release_cached_memory(int32_t device) {
    rpf::cache_release(device);
    return RPF_OK;
}
