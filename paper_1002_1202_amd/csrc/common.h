// Internal definitions shared by the HIP sources of the gsc library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/gsc.h"

namespace gsc {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
    gsc_status code;
    Error(gsc_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define GSC_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            throw ::gsc::Error(e_ == hipErrorOutOfMemory ? GSC_E_NOMEM : GSC_E_DEVICE, \
                               std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GSC_REQUIRE(cond, msg)                                                     \
    do {                                                                           \
        if (!(cond)) throw ::gsc::Error(GSC_E_ARG, msg);                           \
    } while (0)

// ------------------------------------------------------------------ complex
template <typename T> struct alignas(2 * sizeof(T)) cpx { T re, im; };
using c64 = cpx<float>;
using c128 = cpx<double>;

template <typename T> __host__ __device__ inline cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T> __host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cpx<T> cdiv(cpx<T> a, cpx<T> b) {
    // Smith's algorithm: avoids overflow in |b|^2
    if (fabs(b.re) >= fabs(b.im)) {
        T r = b.im / b.re, den = b.re + b.im * r;
        return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    }
    T r = b.re / b.im, den = b.re * r + b.im;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
template <typename T> __host__ __device__ inline T cabs2(cpx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ inline T cabs(cpx<T> a) { return hypot(a.re, a.im); }
template <typename T> __host__ __device__ inline bool cfinite(cpx<T> a) { return isfinite(a.re) && isfinite(a.im); }

template <typename To, typename From> __host__ __device__ inline cpx<To> ccast(cpx<From> a) {
    return {static_cast<To>(a.re), static_cast<To>(a.im)};
}

// ------------------------------------------------------------------ device memory
// ------------------------------------------------------------------ device memory
// Every library temporary comes from dev_alloc.  Blocks of at least 64 MiB
// are kept after dev_free (per device, up to a third of its memory) and
// handed to later requests of at most their size and at least half of it:
// freshly mapped device memory is cleared by the amdgpu kernel driver,
// which for the tens of GB of a full-carry solve costs about a second
// whenever the sizes of consecutive calls differ.  Like hipFree, dev_free of such a block waits
// for the device to go idle before the block can be handed out again.
// Cached blocks hold no data the caller can see.
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// Device-to-host copy into caller memory, stream-ordered after the work
// already on `st`; returns when the data is in `dst`.  Copies of 256 MiB and
// more go through pinned staging buffers drained by host threads.
void copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t st);
void host_staging_release();
size_t dev_cache_bytes(int device);   // bytes cached for this device
size_t dev_usable_bytes();            // free device memory plus this device's cache
void dev_cache_release();             // hand every cached block back

template <typename T> struct DevBuf {
    T *ptr = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), n(o.n) { o.ptr = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); ptr = o.ptr; n = o.n; o.ptr = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count) ptr = static_cast<T *>(dev_alloc(count * sizeof(T)));
        n = count;
    }
    void release() {
        if (ptr) dev_free(ptr);
        ptr = nullptr;
        n = 0;
    }
    T *get() const { return ptr; }
};

// ------------------------------------------------------------------ kernel timing
enum KernelId : int {
    KP_SPMM_SEED = 0, KP_SPMM_S, KP_SHIFT_UPDATE, KP_CG_UPDATE, KP_CG_DIR, KP_UPDATE_R,
    KP_RHO_DOT, KP_P_UPDATE, KP_CTRL, KP_POST, KP_PROJ_UPDATE, KP_CHEB, KP_RING_T,
    KP_LZ_HPROD, KP_LZ_UPDATE, KP_LZ_SCALE, KP_CHEB_MX, KP_MX_RESID, KP_COUNT
};
const char *kernel_name(int id);

// Events recorded around launches while enabled; resolved at sync points.
struct Profiler {
    bool on = false;
    int only = -1;      // time only this kernel id (-1: all)
    struct Acc { double ms = 0; long long launches = 0; double bytes = 0; };
    Acc acc[KP_COUNT];
    struct Pending { int id; hipEvent_t a, b; double bytes; long long launches; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get_event();
    // one launch of kernel id between begin and end
    void begin(hipStream_t st, int id, double bytes) { begin_group(st, id); end_pending_ = {bytes, 1}; }
    void end(hipStream_t st) { end_group(st, end_pending_.launches, end_pending_.bytes); }
    // `launches` back-to-back launches of kernel id between begin_group and
    // end_group, timed by one event pair (their average includes the gaps
    // between them)
    void begin_group(hipStream_t st, int id);
    void end_group(hipStream_t st, long long launches, double bytes);
    void resolve();     // call after the stream was synchronised
    void add_bytes(int id, double bytes) { acc[id].bytes += bytes; }
    void reset();
    ~Profiler();
    bool open_ = false;
    int open_id_ = -1;
    struct { double bytes; long long launches; } end_pending_{0.0, 1};
};

// ------------------------------------------------------------------ handles
struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    Profiler prof;
    void *scratch = nullptr;    // device address of the allocation-free scratch array
};

struct Pair {
    Ctx *ctx = nullptr;
    int device = 0;             // the context's device (destruction does not read ctx)
    int B = 4;
    int64_t nb = 0, n = 0, nnzb = 0;
    DevBuf<int32_t> rowptr;     // nb+1
    DevBuf<int32_t> colidx;     // nnzb
    DevBuf<int32_t> brow;       // nnzb: block row of every stored block
    DevBuf<int32_t> mirror;     // nnzb: index of the stored block (J, I)
    DevBuf<double> H, S;        // nnzb*B*B, FP64
    DevBuf<float> H32, S32;     // FP32 copies for mixed precision products
    bool f32_valid = false;
    std::vector<int64_t> h_rowptr;  // host copies of the pattern
    std::vector<int32_t> h_colidx;
};

// launch geometry: 4 waves of 64 lanes; one wave covers 64 right-hand sides
constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

inline int div_up(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

void ensure_f32(Pair &p);


}  // namespace gsc
