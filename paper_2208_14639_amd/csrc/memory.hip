// Device memory for plans and workspaces: a per-device caching allocator.
//
// Plans are created and destroyed at high rates (one per molecule in the
// benchmark loop, one per request in the server), and hipMalloc/hipFree cost
// tens to hundreds of microseconds each (hipFree synchronises the device).
// Freed blocks are therefore kept per device, sorted by size, and handed to
// later requests of a similar size (a block is reused for requests between
// half its size and its size).  Callers free blocks only after the work that
// used them has completed (vv10_destroy synchronises the plan's stream
// first), so a cached block is never in use when it is handed out again.
// When hipMalloc reports out-of-memory, the device's cached blocks are
// released and the allocation retried once.  The cache holds at most
// VV10_CACHE_BYTES bytes per device (default 64 GiB).
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr size_t kGranule = 256 * 1024;

struct DeviceCache {
    std::multimap<size_t, void *> free_blocks;     // size -> block
    std::unordered_map<void *, size_t> live;        // block -> size
    size_t cached = 0;
};

std::mutex g_mu;
std::map<int, DeviceCache> g_cache;

size_t cache_limit() {
    static const size_t lim = [] {
        const char *s = std::getenv("VV10_CACHE_BYTES");
        return s ? (size_t)std::strtoull(s, nullptr, 10) : (size_t)64 << 30;
    }();
    return lim;
}

size_t round_size(size_t n) {
    if (n == 0) n = 1;
    // granule of 1/8 of the size's power of two (at least 256 KiB): <= 12.5% slack
    size_t p = 1;
    while (p < n) p <<= 1;
    size_t g = std::max(kGranule, p >> 3);
    return (n + g - 1) / g * g;
}

void release_all(DeviceCache &c) {
    for (auto &kv : c.free_blocks) (void)hipFree(kv.second);
    c.free_blocks.clear();
    c.cached = 0;
}

}  // namespace

hipError_t dev_alloc(void **ptr, size_t bytes) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t n = round_size(bytes);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCache &c = g_cache[dev];
        auto it = c.free_blocks.lower_bound(n);
        if (it != c.free_blocks.end() && it->first <= 2 * n) {
            *ptr = it->second;
            c.live[it->second] = it->first;
            c.cached -= it->first;
            c.free_blocks.erase(it);
            return hipSuccess;
        }
    }
    e = hipMalloc(ptr, n);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_mu);
            release_all(g_cache[dev]);
        }
        e = hipMalloc(ptr, n);
    }
    if (e != hipSuccess) {
        *ptr = nullptr;
        return e;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[dev].live[*ptr] = n;
    return hipSuccess;
}

void dev_free(void *ptr) {
    if (!ptr) return;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_cache) {
        DeviceCache &c = kv.second;
        auto it = c.live.find(ptr);
        if (it == c.live.end()) continue;
        const size_t n = it->second;
        c.live.erase(it);
        if (c.cached + n <= cache_limit()) {
            c.free_blocks.emplace(n, ptr);
            c.cached += n;
        } else {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(kv.first);
            (void)hipFree(ptr);
            (void)hipSetDevice(cur);
        }
        return;
    }
    (void)hipFree(ptr);   // not from this allocator
}

size_t dev_cached_bytes() {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t t = 0;
    for (auto &kv : g_cache) t += kv.second.cached;
    return t;
}

void dev_release_cached() {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_cache) {
        (void)hipSetDevice(kv.first);
        release_all(kv.second);
    }
    (void)hipSetDevice(cur);
}

}  // namespace vv10

extern "C" {

size_t vv10_cached_bytes(void) { return vv10::dev_cached_bytes(); }

void vv10_release_cached(void) { vv10::dev_release_cached(); }

}  // extern "C"
