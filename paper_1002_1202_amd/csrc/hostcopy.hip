// Bulk device-to-host copies into caller (pageable) memory through pinned
// staging buffers: the copy engine fills the next buffers while host
// threads drain a filled one into the destination, so the PCIe transfer,
// the host-side copy and the first touch of the destination pages overlap.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace gsc {

namespace {

constexpr size_t kStage = size_t(256) << 20;   // bytes per staging buffer
constexpr int kNStage = 3;                      // buffers in flight
constexpr int kDrainThreads = 8;

struct Staging {
    std::mutex m;
    void *buf[kNStage] = {};
    hipEvent_t ev[kNStage] = {};
    bool ready = false;
};

Staging &staging() {
    static Staging *s = new Staging;   // released by host_staging_release
    return *s;
}

// copy `len` bytes with up to kDrainThreads threads (each a contiguous part)
void parallel_copy(char *dst, const char *src, size_t len) {
    const int nt = static_cast<int>(std::min<size_t>(kDrainThreads, std::max<size_t>(1, len >> 24)));
    if (nt <= 1) {
        std::memcpy(dst, src, len);
        return;
    }
    const size_t part = (len + nt - 1) / nt;
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        const size_t o = std::min(len, static_cast<size_t>(t) * part);
        const size_t l = std::min(len - o, part);
        try {
            th.emplace_back([=] { std::memcpy(dst + o, src + o, l); });
        } catch (...) {
            std::memcpy(dst + o, src + o, l);   // no thread available: copy this part here
        }
    }
    for (auto &x : th) x.join();
}

// the caller holds the lock
bool ensure_staging(Staging &S) {
    if (S.ready) return true;
    for (int i = 0; i < kNStage; ++i) {
        if (hipHostMalloc(&S.buf[i], kStage, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&S.ev[i], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j <= i; ++j) {
                if (S.buf[j]) (void)hipHostFree(S.buf[j]);
                if (S.ev[j]) (void)hipEventDestroy(S.ev[j]);
                S.buf[j] = nullptr;
                S.ev[j] = nullptr;
            }
            return false;
        }
    }
    S.ready = true;
    return true;
}

}  // namespace

void copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return;
    Staging &S = staging();
    std::unique_lock<std::mutex> lk(S.m, std::defer_lock);
    if (bytes >= kStage) lk.lock();
    if (bytes < kStage || !ensure_staging(S)) {
        // small copies (or no pinned memory): the runtime's own path
        GSC_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        GSC_HIP(hipStreamSynchronize(st));
        return;
    }
    const char *s = static_cast<const char *>(src);
    char *d = static_cast<char *>(dst);
    const size_t nchunk = (bytes + kStage - 1) / kStage;
    auto enqueue = [&](size_t c) {
        const int b = static_cast<int>(c % kNStage);
        const size_t off = c * kStage, len = std::min(kStage, bytes - off);
        GSC_HIP(hipMemcpyAsync(S.buf[b], s + off, len, hipMemcpyDeviceToHost, st));
        GSC_HIP(hipEventRecord(S.ev[b], st));
    };
    for (size_t c = 0; c < std::min<size_t>(kNStage, nchunk); ++c) enqueue(c);
    for (size_t c = 0; c < nchunk; ++c) {
        const int b = static_cast<int>(c % kNStage);
        const size_t off = c * kStage, len = std::min(kStage, bytes - off);
        GSC_HIP(hipEventSynchronize(S.ev[b]));
        parallel_copy(d + off, static_cast<const char *>(S.buf[b]), len);
        if (c + kNStage < nchunk) enqueue(c + kNStage);
    }
}

void host_staging_release() {
    Staging &S = staging();
    std::lock_guard<std::mutex> lk(S.m);
    if (!S.ready) return;
    for (int i = 0; i < kNStage; ++i) {
        (void)hipEventSynchronize(S.ev[i]);
        (void)hipHostFree(S.buf[i]);
        (void)hipEventDestroy(S.ev[i]);
        S.buf[i] = nullptr;
        S.ev[i] = nullptr;
    }
    S.ready = false;
}

}  // namespace gsc
