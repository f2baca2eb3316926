// Cache of large device blocks behind DevBuf (dev_alloc / dev_free).
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.h"

namespace gsc {

namespace {

constexpr size_t kCacheMin = size_t(64) << 20;   // smaller blocks go straight to the runtime

struct Pool {
    std::mutex m;
    std::unordered_map<void *, std::pair<size_t, int>> live;   // large blocks in use: size, device
    std::multimap<std::pair<int, size_t>, void *> free;         // cached blocks by (device, size)
    std::map<int, size_t> cached;                               // cached bytes per device
    std::map<int, size_t> limit;                                // cache limit per device
};

Pool &pool() {
    static Pool *p = new Pool;   // never destroyed: cached blocks die with the process
    return *p;
}

// hand the cached blocks of one device (or every device, dev < 0) back; the
// caller holds the lock
void release_locked(Pool &P, int dev) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto it = P.free.begin(); it != P.free.end();) {
        if (dev >= 0 && it->first.first != dev) { ++it; continue; }
        (void)hipSetDevice(it->first.first);
        (void)hipFree(it->second);
        P.cached[it->first.first] -= it->first.second;
        it = P.free.erase(it);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
}

}  // namespace

void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    if (bytes < kCacheMin) {
        GSC_HIP(hipMalloc(&p, bytes));
        return p;
    }
    int dev = 0;
    GSC_HIP(hipGetDevice(&dev));
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> lk(P.m);
        auto it = P.free.lower_bound({dev, bytes});
        if (it != P.free.end() && it->first.first == dev && it->first.second / 2 <= bytes) {
            p = it->second;
            const size_t sz = it->first.second;
            P.free.erase(it);
            P.cached[dev] -= sz;
            P.live[p] = {sz, dev};
            return p;
        }
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        // out of memory with blocks cached: give them back and try once more
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(P.m);
            release_locked(P, dev);
        }
        GSC_HIP(hipMalloc(&p, bytes));
    }
    std::lock_guard<std::mutex> lk(P.m);
    P.live[p] = {bytes, dev};
    return p;
}

void dev_free(void *p) {
    if (p == nullptr) return;
    Pool &P = pool();
    size_t sz = 0;
    int dev = -1;
    {
        std::lock_guard<std::mutex> lk(P.m);
        auto it = P.live.find(p);
        if (it != P.live.end()) {
            sz = it->second.first;
            dev = it->second.second;
            P.live.erase(it);
            if (P.limit.find(dev) == P.limit.end()) {
                size_t freeb = 0, totalb = 0;
                int cur = -1;
                (void)hipGetDevice(&cur);
                (void)hipSetDevice(dev);
                if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) totalb = 0;
                if (cur >= 0) (void)hipSetDevice(cur);
                P.limit.emplace(dev, totalb / 3);
            }
            if (P.cached[dev] + sz > P.limit[dev]) dev = -1;
        }
    }
    if (dev >= 0) {
        // hipFree waits for the device to go idle; a cached block has to as
        // well, or a call on another stream could receive it while kernels
        // still use it (the wait runs outside the lock)
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != dev) (void)hipSetDevice(dev);
        const bool idle = hipDeviceSynchronize() == hipSuccess;
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        if (idle) {
            std::lock_guard<std::mutex> lk(P.m);
            if (P.cached[dev] + sz <= P.limit[dev]) {
                P.free.insert({{dev, sz}, p});
                P.cached[dev] += sz;
                return;
            }
        }
    }
    (void)hipFree(p);
}

size_t dev_cache_bytes(int device) {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.m);
    auto it = P.cached.find(device);
    return it == P.cached.end() ? 0 : it->second;
}

size_t dev_usable_bytes() {
    size_t freeb = 0, totalb = 0;
    GSC_HIP(hipMemGetInfo(&freeb, &totalb));
    int dev = 0;
    GSC_HIP(hipGetDevice(&dev));
    return freeb + dev_cache_bytes(dev);
}

void dev_cache_release() {
    {
        Pool &P = pool();
        std::lock_guard<std::mutex> lk(P.m);
        release_locked(P, -1);
    }
    host_staging_release();
}

}  // namespace gsc
