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
        n = count;
        if (count) GSC_HIP(hipMalloc(&ptr, count * sizeof(T)));
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        n = 0;
    }
    T *get() const { return ptr; }
};

// ------------------------------------------------------------------ handles
struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
};

struct Pair {
    Ctx *ctx = nullptr;
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
