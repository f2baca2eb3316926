// C ABI of the gsc library: argument validation, error mapping and the
// reductions to Mulliken charges and band energy (Sec. 2.2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "csc.h"
#include "pair.h"
#include "solver.h"
#include "spmm.h"

struct gsc_ctx { gsc::Ctx c; };
struct gsc_pair { gsc::Pair p; };
struct gsc_csc { gsc::Csc c; };

namespace gsc {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }

template <typename F> gsc_status guarded(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return GSC_E_NOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return GSC_E_DEVICE;
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) GSC_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// q_a = -(2/pi) sum_k w_k Im sg_ka ; e_a = -(2/pi) sum_k w_k E_k Im sg_ka
__global__ void k_mulliken(int K, int R, const c128 *sg, size_t ld_k, size_t ld_r, const c128 *z,
                           const double *w, double *q, double *e) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double aq = 0.0, ae = 0.0;
    for (int k = 0; k < K; ++k) {
        const double im = sg[static_cast<size_t>(k) * ld_k + static_cast<size_t>(r) * ld_r].im;
        aq += w[k] * im;
        ae += w[k] * z[k].re * im;
    }
    const double f = -2.0 / M_PI;
    q[r] = f * aq;
    e[r] = f * ae;
}

// t_k = sum_a Im (S G_k)_aa over the R orbitals of shift k (one block per k)
__global__ void k_sg_trace(int R, const c128 *sg, double *t) {
    __shared__ double lds[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int a = threadIdx.x; a < R; a += 256) s += sg[static_cast<size_t>(k) * R + a].im;
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) t[k] = lds[0];
}

// Trapezoid weights over the ascending grid E truncated at ef, with the
// integrand linear between samples: sum_k w_k f(E_k) is the integral of the
// interpolant from E_0 to ef.
void truncated_trapezoid(const std::vector<double> &E, double ef, std::vector<double> &w) {
    const size_t K = E.size();
    w.assign(K, 0.0);
    for (size_t j = 0; j + 1 < K && ef > E[j]; ++j) {
        const double h = E[j + 1] - E[j];
        const double d = std::min(ef - E[j], h);
        w[j] += d - 0.5 * d * d / h;
        w[j + 1] += 0.5 * d * d / h;
    }
}

double electron_count(const std::vector<double> &E, const std::vector<double> &t, double ef,
                      std::vector<double> &w) {
    truncated_trapezoid(E, ef, w);
    double s = 0.0;
    for (size_t k = 0; k < E.size(); ++k) s += w[k] * t[k];
    return -2.0 / M_PI * s;
}

__global__ void k_sum(int n, const double *v, double *out) {
    __shared__ double lds[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) lds[threadIdx.x] += lds[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = lds[0];
}

// Band-energy gradient on the stored entries from the weighted accumulators
// of column c (projection m at pattern row b):
//   dE/dH_bc = -(2/pi) sum_k w_k E_k Im (G S G)_bc = (2/pi) Im AD
//   dE/dS_bc = -(2/pi) sum_k w_k E_k Im (G - z G S G)_bc = -(2/pi) Im (AG + AZ)
// (G S G e_c = -dx/dz); e_c = -(2/pi) Im AG of the S e_c projection.
__global__ void k_vjp_assemble(int R, int M, const c128 *acc, const int64_t *vidx, double grad_E, double *dH,
                               double *dS, double *e_col) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(R) * M) return;
    const int c = static_cast<int>(t / M), m = static_cast<int>(t % M);
    const c128 *A = acc + static_cast<size_t>(t) * 3;
    const double f = 2.0 / M_PI;
    if (m == M - 1) {
        e_col[c] = -f * A[0].im;
        return;
    }
    const int64_t v = vidx[t];
    if (v < 0) return;
    dH[v] += grad_E * f * A[1].im;
    dS[v] += grad_E * (-f) * (A[0].im + A[2].im);
}

__global__ void k_pad_cols(int N, int R, int Rp, const c128 *in, c128 *out, int to_padded) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * Rp) return;
    const int64_t i = t / Rp;
    const int c = static_cast<int>(t % Rp);
    if (to_padded) out[t] = c < R ? in[i * R + c] : c128{0, 0};
    else if (c < R) out[i * R + c] = in[t];
}

// ------------------------------------------------------------------ allocation-free product
// gsc_spmm_noalloc works in this fixed array instead of allocating: one copy
// per device, part of the code object, held until the process ends.  In host
// code the name is only a host-side stand-in, never a device address: host
// code uses the address hipGetSymbolAddress returns, fetched once per device
// (with that device current) when a context is created, and kept in the
// context.
constexpr size_t kScratchBytes = size_t{64} << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on `device`, which must be the current device.
void *scratch_address(int device) {
    static std::mutex mu;
    static void *addr[64] = {};
    GSC_REQUIRE(device >= 0 && device < 64, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (addr[device] == nullptr) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            throw Error(GSC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[device] = ptr;
    }
    return addr[device];
}

// per-column shift index c and zero shifts for the padding columns c >= R
__global__ void k_noalloc_cols(int R, int Rp, c128 *z, int *seed) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Rp) return;
    seed[c] = c;
    if (c >= R) z[c] = c128{0.0, 0.0};
}

// (S G_k)_aa for the unit right-hand sides e_a, a = orb_idx[r], into the
// device array sg [nshift][norb]: the projected solve carrying c = S e_a,
// or the full carry's columns projected on S e_a.
gsc_status sg_solve(Ctx &ctx, const Pair &p, int nshift, const double *z, int norb, const int64_t *orb_idx,
                    const gsc_opts &o, c128 *sg, gsc_stats *stats) {
    SolveRequest req;
    req.pair = &p;
    req.K = nshift;
    req.z = z;
    req.R = norb;
    req.rhs_idx = orb_idx;
    req.opts = o;
    req.out_mem = GSC_MEM_DEVICE;
    req.stats = stats;
    ProjSpec ps;
    if (o.carry == GSC_CARRY_FULL) {
        req.sg_diag = sg;
    } else {
        ps.M = 0;
        ps.srow = true;
        req.proj = &ps;
        req.proj_out = sg;
    }
    return run_solve(ctx, req);
}

void validate_opts(const gsc_opts &o) {
    GSC_REQUIRE(o.tol > 0 && std::isfinite(o.tol), "tol must be positive");
    GSC_REQUIRE(o.max_iter > 0, "max_iter must be positive");
    GSC_REQUIRE(o.inner_max_iter > 0, "inner_max_iter must be positive");
    GSC_REQUIRE(o.precision == GSC_FP64 || o.precision == GSC_MIXED || o.precision == GSC_C64, "unknown precision");
    GSC_REQUIRE(o.carry == GSC_CARRY_FULL || o.carry == GSC_CARRY_PROJECTED, "unknown carry mode");
    GSC_REQUIRE(o.fuse_steps >= 0 && o.fuse_steps <= kMaxFuse, "fuse_steps must be in [0, 16]");
    GSC_REQUIRE(o.spmm_kernel >= 0 && o.spmm_kernel <= 1, "spmm_kernel must be 0 or 1");
    GSC_REQUIRE(o.stream_hint >= 0 && o.stream_hint <= 2, "stream_hint must be 0, 1 or 2");
    GSC_REQUIRE(o.cheb_block >= 0 && o.cheb_block % 64 == 0, "cheb_block must be 0 or a multiple of 64");
    GSC_REQUIRE(o.inner_relax == 0 || o.inner_relax == 1, "inner_relax must be 0 or 1");
    GSC_REQUIRE(o.inner_method >= 0 && o.inner_method <= 2, "inner_method must be 0, 1 or 2");
    GSC_REQUIRE(o.row_groups >= 0 && o.row_groups % 8 == 0 && o.row_groups <= 65528,
                "row_groups must be 0 or a multiple of 8 up to 65528");
    GSC_REQUIRE(o.batch_mem_mb >= 0, "batch_mem_mb must not be negative");
}

void validate_shifts(int nshift, const double *z, int seed_index) {
    GSC_REQUIRE(nshift >= 1 && z != nullptr, "need at least one shift");
    GSC_REQUIRE(nshift <= 65535, "at most 65535 shifts per call");
    for (int k = 0; k < nshift; ++k) {
        GSC_REQUIRE(std::isfinite(z[2 * k]) && std::isfinite(z[2 * k + 1]), "shifts must be finite");
        GSC_REQUIRE(z[2 * k + 1] > 0.0, "every shift needs Im z > 0 (z S - H must be nonsingular)");
    }
    GSC_REQUIRE(seed_index < nshift, "seed_index out of range");
}

}  // namespace gsc

using namespace gsc;

extern "C" {

void gsc_opts_default(gsc_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->max_iter = 5000;
    o->inner_tol = 0.0;
    o->inner_max_iter = 200;
    o->precision = GSC_FP64;
    o->carry = GSC_CARRY_FULL;
    o->seed_index = -1;
    o->fuse_steps = 0;
    o->rhs_tile = 0;
    o->recheck = 0;
}

const char *gsc_last_error(void) { return g_last_error.c_str(); }
const char *gsc_version(void) { return "gsc 0.1 (gfx950)"; }

gsc_status gsc_create(gsc_ctx **out, int device, void *stream) {
    return guarded([&] {
        GSC_REQUIRE(out != nullptr, "out must not be NULL");
        int n = 0;
        GSC_HIP(hipGetDeviceCount(&n));
        GSC_REQUIRE(device >= 0 && device < n, "device ordinal out of range");
        auto c = std::make_unique<gsc_ctx>();
        c->c.device = device;
        c->c.stream = static_cast<hipStream_t>(stream);
        DeviceGuard g(device);
        hipDeviceProp_t prop;
        GSC_HIP(hipGetDeviceProperties(&prop, device));
        c->c.num_cu = prop.multiProcessorCount;
        c->c.scratch = scratch_address(device);
        *out = c.release();
        return GSC_OK;
    });
}

gsc_status gsc_set_stream(gsc_ctx *ctx, void *stream) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr, "ctx must not be NULL");
        ctx->c.stream = static_cast<hipStream_t>(stream);
        return GSC_OK;
    });
}

void gsc_destroy(gsc_ctx *ctx) {
    delete ctx;
    dev_cache_release();
}

gsc_status gsc_release_cache(void) {
    return guarded([&] {
        dev_cache_release();
        return GSC_OK;
    });
}

gsc_status gsc_pair_create(gsc_ctx *ctx, int block, int64_t nbrows, const int64_t *rowptr,
                           const int32_t *colidx, const double *Hval, const double *Sval, int mem,
                           gsc_pair **out) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && out != nullptr, "ctx/out must not be NULL");
        DeviceGuard g(ctx->c.device);
        auto p = std::make_unique<gsc_pair>();
        p->p.ctx = &ctx->c;
        p->p.device = ctx->c.device;
        validate_and_upload(p->p, block, nbrows, rowptr, colidx);
        if (Hval || Sval) set_values(p->p, Hval, Sval, mem);
        *out = p.release();
        return GSC_OK;
    });
}

gsc_status gsc_pair_set_values(gsc_pair *pair, const double *Hval, const double *Sval, int mem) {
    return guarded([&] {
        GSC_REQUIRE(pair != nullptr, "pair must not be NULL");
        DeviceGuard g(pair->p.ctx->device);
        set_values(pair->p, Hval, Sval, mem);
        return GSC_OK;
    });
}

gsc_status gsc_pair_get_values(const gsc_pair *pair, double *Hval, double *Sval, int mem) {
    return guarded([&] {
        GSC_REQUIRE(pair != nullptr, "pair must not be NULL");
        const Pair &p = pair->p;
        DeviceGuard g(p.ctx->device);
        const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
        const hipMemcpyKind kind = mem == GSC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (Hval) GSC_HIP(hipMemcpyAsync(Hval, p.H.get(), nv * 8, kind, p.ctx->stream));
        if (Sval) GSC_HIP(hipMemcpyAsync(Sval, p.S.get(), nv * 8, kind, p.ctx->stream));
        GSC_HIP(hipStreamSynchronize(p.ctx->stream));
        return GSC_OK;
    });
}

gsc_status gsc_pair_info(const gsc_pair *pair, int64_t *n, int64_t *nnzb, int *block) {
    return guarded([&] {
        GSC_REQUIRE(pair != nullptr, "pair must not be NULL");
        if (n) *n = pair->p.n;
        if (nnzb) *nnzb = pair->p.nnzb;
        if (block) *block = pair->p.B;
        return GSC_OK;
    });
}

// destruction reads the device ordinal kept in the object, never the
// context, which may already be gone
void gsc_pair_destroy(gsc_pair *pair) {
    if (!pair) return;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    const int dev = pair->p.device;
    if (prev != dev) (void)hipSetDevice(dev);
    delete pair;
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

gsc_status gsc_ased_build(gsc_ctx *ctx, const gsc_ased_geom *geom, double scale, gsc_pair *pair,
                          double *scale_out) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        DeviceGuard g(ctx->c.device);
        const double c = ased_build(pair->p, geom, scale);
        if (!(std::isfinite(c) && c > 0)) throw Error(GSC_E_NAN, "ASED scale is not finite");
        if (scale_out) *scale_out = c;
        return GSC_OK;
    });
}

gsc_status gsc_ased_vjp(gsc_ctx *ctx, const gsc_ased_geom *geom, double scale, const gsc_pair *pair,
                        const double *dHval, const double *dSval, int mem, double *forces) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        DeviceGuard g(ctx->c.device);
        ased_vjp(pair->p, geom, scale, dHval, dSval, mem, forces);
        return GSC_OK;
    });
}

gsc_status gsc_spmm(gsc_ctx *ctx, const gsc_pair *pair, int nrhs, const double *alpha_S, const double *X,
                    double *Y, int mem) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        GSC_REQUIRE(nrhs > 0 && alpha_S && X && Y, "bad spmm arguments");
        DeviceGuard g(ctx->c.device);
        const Pair &p = pair->p;
        hipStream_t st = ctx->c.stream;
        const int N = static_cast<int>(p.n);
        const int Rp = (nrhs + 63) / 64 * 64;
        DevBuf<c128> xin, xp(static_cast<size_t>(N) * Rp), yp(static_cast<size_t>(N) * Rp), yout;
        const c128 *src = reinterpret_cast<const c128 *>(X);
        if (mem != GSC_MEM_DEVICE) {
            xin.alloc(static_cast<size_t>(N) * nrhs);
            GSC_HIP(hipMemcpyAsync(xin.get(), X, xin.n * sizeof(c128), hipMemcpyHostToDevice, st));
            src = xin.get();
        }
        const int64_t tot = static_cast<int64_t>(N) * Rp;
        k_pad_cols<<<div_up(tot, 256), 256, 0, st>>>(N, nrhs, Rp, src, xp.get(), 1);
        std::vector<c128> za(Rp, c128{0, 0});
        std::vector<int> iota(Rp);
        for (int c = 0; c < Rp; ++c) iota[c] = c;
        for (int c = 0; c < nrhs; ++c) za[c] = c128{alpha_S[2 * c], alpha_S[2 * c + 1]};
        DevBuf<c128> dz(Rp);
        DevBuf<int> dseed(Rp);
        GSC_HIP(hipMemcpyAsync(dz.get(), za.data(), Rp * sizeof(c128), hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(dseed.get(), iota.data(), Rp * sizeof(int), hipMemcpyHostToDevice, st));
        TileDims td{};
        td.N = N; td.nb = static_cast<int>(p.nb); td.B = p.B; td.Rp = Rp;
        set_spmm_geometry(td, p);
        DevBuf<c128> part(static_cast<size_t>(td.Gs) * Rp);
        launch_spmm_seed<double>(st, p, td, p.S.get(), p.H.get(), xp.get(), yp.get(), dz.get(), dseed.get(),
                                 nullptr, part.get());
        c128 *dst = reinterpret_cast<c128 *>(Y);
        if (mem != GSC_MEM_DEVICE) {
            yout.alloc(static_cast<size_t>(N) * nrhs);
            dst = yout.get();
        }
        k_pad_cols<<<div_up(tot, 256), 256, 0, st>>>(N, nrhs, Rp, yp.get(), dst, 0);
        GSC_HIP(hipGetLastError());
        if (mem != GSC_MEM_DEVICE)
            GSC_HIP(hipMemcpyAsync(Y, yout.get(), yout.n * sizeof(c128), hipMemcpyDeviceToHost, st));
        GSC_HIP(hipStreamSynchronize(st));
        return GSC_OK;
    });
}

gsc_status gsc_spmm_noalloc(gsc_ctx *ctx, const gsc_pair *pair, int nrhs, const double *alpha_S, const double *X,
                            double *Y) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        GSC_REQUIRE(nrhs > 0 && alpha_S && X && Y, "bad spmm arguments");
        GSC_REQUIRE(ctx->c.scratch != nullptr, "the context has no scratch address");
        DeviceGuard g(ctx->c.device);
        const Pair &p = pair->p;
        hipStream_t st = ctx->c.stream;
        const int N = static_cast<int>(p.n);
        const int Rp = (nrhs + 63) / 64 * 64;
        TileDims td{};
        td.N = N; td.nb = static_cast<int>(p.nb); td.B = p.B; td.Rp = Rp;
        set_spmm_geometry(td, p);
        // the scratch: shifts [Rp], seed indices [Rp], partial dots [Gs][Rp]
        // and, unless nrhs is a multiple of 64, padded copies of X and Y
        const bool direct = Rp == nrhs;
        size_t off = 0;
        auto carve = [&off](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) / 256 * 256;
            return o;
        };
        const size_t NRp = static_cast<size_t>(N) * Rp;
        const size_t oz = carve(Rp * sizeof(c128));
        const size_t os = carve(Rp * sizeof(int));
        const size_t op = carve(static_cast<size_t>(td.Gs) * Rp * sizeof(c128));
        const size_t ox = direct ? 0 : carve(NRp * sizeof(c128));
        const size_t oy = direct ? 0 : carve(NRp * sizeof(c128));
        if (off > kScratchBytes)
            throw Error(GSC_E_ARG, "gsc_spmm_noalloc needs " + std::to_string(off) +
                                       " bytes of scratch, more than its maximum of " +
                                       std::to_string(kScratchBytes) + " (fewer rhs or a multiple of 64)");
        unsigned char *base = static_cast<unsigned char *>(ctx->c.scratch);
        c128 *dz = reinterpret_cast<c128 *>(base + oz);
        int *dseed = reinterpret_cast<int *>(base + os);
        c128 *part = reinterpret_cast<c128 *>(base + op);
        GSC_HIP(hipMemcpyAsync(dz, alpha_S, static_cast<size_t>(nrhs) * sizeof(c128), hipMemcpyHostToDevice, st));
        k_noalloc_cols<<<div_up(Rp, 256), 256, 0, st>>>(nrhs, Rp, dz, dseed);
        const c128 *xin = reinterpret_cast<const c128 *>(X);
        c128 *yout = reinterpret_cast<c128 *>(Y);
        if (!direct) {
            c128 *xp = reinterpret_cast<c128 *>(base + ox);
            k_pad_cols<<<div_up(static_cast<int64_t>(NRp), 256), 256, 0, st>>>(N, nrhs, Rp, xin, xp, 1);
            xin = xp;
            yout = reinterpret_cast<c128 *>(base + oy);
        }
        launch_spmm_seed<double>(st, p, td, p.S.get(), p.H.get(), xin, yout, dz, dseed, nullptr, part);
        if (!direct)
            k_pad_cols<<<div_up(static_cast<int64_t>(NRp), 256), 256, 0, st>>>(N, nrhs, Rp, yout,
                                                                               reinterpret_cast<c128 *>(Y), 0);
        GSC_HIP(hipGetLastError());
        GSC_HIP(hipStreamSynchronize(st));
        return GSC_OK;
    });
}

gsc_status gsc_solve(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, int nrhs,
                     const int64_t *rhs_idx, const double *B_dense, const gsc_opts *opts, double *G_cols,
                     int nproj, const int64_t *proj_idx, double *G_proj, int out_mem, gsc_stats *stats) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        validate_opts(o);
        validate_shifts(nshift, z, o.seed_index);
        const Pair &p = pair->p;
        GSC_REQUIRE(nrhs >= 1, "need at least one right-hand side");
        GSC_REQUIRE(rhs_idx != nullptr || B_dense != nullptr, "rhs_idx or B_dense is required");
        if (rhs_idx)
            for (int r = 0; r < nrhs; ++r) GSC_REQUIRE(rhs_idx[r] >= 0 && rhs_idx[r] < p.n, "rhs index out of range");
        GSC_REQUIRE(nproj >= 0, "nproj must be >= 0");
        if (nproj > 0) {
            GSC_REQUIRE(proj_idx != nullptr && G_proj != nullptr, "proj_idx and G_proj are required when nproj > 0");
            for (int64_t t = 0; t < static_cast<int64_t>(nrhs) * nproj; ++t)
                GSC_REQUIRE(proj_idx[t] >= 0 && proj_idx[t] < p.n, "projection index out of range");
        }
        if (o.carry == GSC_CARRY_PROJECTED) {
            GSC_REQUIRE(G_cols == nullptr, "G_cols needs the full carry");
            GSC_REQUIRE(nproj > 0, "the projected carry needs projections");
            GSC_REQUIRE(nproj <= 1024, "at most 1024 projections per rhs");
        }
        DeviceGuard g(ctx->c.device);
        SolveRequest req;
        req.pair = &p;
        req.K = nshift;
        req.z = z;
        req.R = nrhs;
        req.rhs_idx = rhs_idx;
        req.B_dense = B_dense;
        req.opts = o;
        req.G_cols = G_cols;
        req.out_mem = out_mem;
        req.stats = stats;
        ProjSpec ps;
        DevBuf<c128> pout;
        if (o.carry == GSC_CARRY_FULL) {
            req.nproj = nproj;
            req.proj_idx = proj_idx;
            req.G_proj = G_proj;
        } else {
            ps.M = nproj;
            ps.srow = false;
            ps.idx.resize(static_cast<size_t>(nrhs) * nproj);
            for (size_t t = 0; t < ps.idx.size(); ++t) ps.idx[t] = static_cast<int32_t>(proj_idx[t]);
            req.proj = &ps;
            if (out_mem == GSC_MEM_DEVICE) {
                req.proj_out = reinterpret_cast<c128 *>(G_proj);
            } else {
                pout.alloc(static_cast<size_t>(nshift) * nrhs * nproj);
                req.proj_out = pout.get();
            }
        }
        const gsc_status s = run_solve(ctx->c, req);
        if (pout.get()) {
            GSC_HIP(hipMemcpyAsync(G_proj, pout.get(), pout.n * sizeof(c128), hipMemcpyDeviceToHost, ctx->c.stream));
        }
        GSC_HIP(hipStreamSynchronize(ctx->c.stream));
        return s;
    });
}

gsc_status gsc_lanczos_green(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, int nrhs,
                             const int64_t *rhs_idx, int m_max, double tol, int check_every,
                             const gsc_opts *opts, double *G_diag, double *coef_a, double *coef_b,
                             int *steps, int out_mem, gsc_stats *stats) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        validate_opts(o);
        validate_shifts(nshift, z, -1);
        const Pair &p = pair->p;
        GSC_REQUIRE(nrhs >= 1 && rhs_idx != nullptr, "need at least one right-hand side index");
        for (int r = 0; r < nrhs; ++r) GSC_REQUIRE(rhs_idx[r] >= 0 && rhs_idx[r] < p.n, "rhs index out of range");
        GSC_REQUIRE(m_max >= 1, "m_max must be >= 1");
        GSC_REQUIRE(check_every >= 0, "check_every must be >= 0");
        GSC_REQUIRE(check_every == 0 || tol > 0.0, "tol must be positive when checks are enabled");
        GSC_REQUIRE(G_diag != nullptr, "G_diag must not be NULL");
        DeviceGuard g(ctx->c.device);
        LanczosRequest req;
        req.pair = &p;
        req.K = nshift;
        req.z = z;
        req.P = nrhs;
        req.rhs_idx = rhs_idx;
        req.m_max = m_max;
        req.tol = tol;
        req.check_every = check_every;
        req.opts = o;
        req.G_diag = G_diag;
        req.coef_a = coef_a;
        req.coef_b = coef_b;
        req.steps = steps;
        req.out_mem = out_mem;
        req.stats = stats;
        return run_lanczos(ctx->c, req);
    });
}

gsc_status gsc_charge_vjp(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, const double *w,
                          int norb, const int64_t *orb_idx, const double *qbar, const gsc_opts *opts,
                          double *dHval, double *dSval, int mem, gsc_stats *stats) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        GSC_REQUIRE(w != nullptr && qbar != nullptr && dHval != nullptr && dSval != nullptr, "NULL argument");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        o.carry = GSC_CARRY_FULL;
        validate_opts(o);
        validate_shifts(nshift, z, o.seed_index);
        const Pair &p = pair->p;
        GSC_REQUIRE(norb >= 1 && orb_idx != nullptr, "need at least one orbital");
        for (int r = 0; r < norb; ++r) GSC_REQUIRE(orb_idx[r] >= 0 && orb_idx[r] < p.n, "orbital index out of range");
        DeviceGuard g(ctx->c.device);
        hipStream_t st = ctx->c.stream;
        const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
        DevBuf<double> dH, dS;
        double *gH = dHval, *gS = dSval;
        if (mem != GSC_MEM_DEVICE) {
            dH.alloc(nv);
            dS.alloc(nv);
            GSC_HIP(hipMemcpyAsync(dH.get(), dHval, nv * 8, hipMemcpyHostToDevice, st));
            GSC_HIP(hipMemcpyAsync(dS.get(), dSval, nv * 8, hipMemcpyHostToDevice, st));
            gH = dH.get();
            gS = dS.get();
        }
        DevBuf<c128> dz(nshift);
        DevBuf<double> dw(nshift);
        GSC_HIP(hipMemcpyAsync(dz.get(), z, nshift * sizeof(c128), hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(dw.get(), w, nshift * sizeof(double), hipMemcpyHostToDevice, st));
        // orbitals per tile: two [K][R][N] complex solution sets in 40 % of free memory
        const size_t freeb = dev_usable_bytes();
        const double per = 2.0 * nshift * static_cast<double>(p.n) * sizeof(c128) + 16.0 * p.n * sizeof(c128);
        int Rt = o.rhs_tile > 0 ? o.rhs_tile : static_cast<int>(0.4 * static_cast<double>(freeb) / per);
        Rt = std::max(1, std::min(Rt, norb));
        bool conv = true;
        long long inner = 0, sri = 0;
        int outer = 0;
        for (int r0 = 0; r0 < norb; r0 += Rt) {
            const int R = std::min(Rt, norb - r0);
            DevBuf<int64_t> dorb(R);
            DevBuf<double> dqb(R);
            GSC_HIP(hipMemcpyAsync(dorb.get(), orb_idx + r0, R * sizeof(int64_t), hipMemcpyHostToDevice, st));
            GSC_HIP(hipMemcpyAsync(dqb.get(), qbar + r0, R * sizeof(double), hipMemcpyHostToDevice, st));
            DevBuf<c128> X(static_cast<size_t>(nshift) * R * p.n), Lm(static_cast<size_t>(nshift) * R * p.n);
            DevBuf<c128> Bs(static_cast<size_t>(R) * p.n);
            launch_s_columns(st, p, R, dorb.get(), Bs.get());
            gsc_stats s1{}, s2{};
            for (int pass = 0; pass < 2; ++pass) {
                SolveRequest req;
                req.pair = &p;
                req.K = nshift;
                req.z = z;
                req.R = R;
                req.opts = o;
                req.out_mem = GSC_MEM_DEVICE;
                req.stats = pass == 0 ? &s1 : &s2;
                if (pass == 0) {
                    req.rhs_idx = orb_idx + r0;
                    req.G_cols = reinterpret_cast<double *>(X.get());
                } else {
                    req.B_dense = reinterpret_cast<const double *>(Bs.get());
                    req.G_cols = reinterpret_cast<double *>(Lm.get());
                }
                const gsc_status s = run_solve(ctx->c, req);
                if (s < 0) return s;
                if (s == GSC_NOT_CONVERGED) conv = false;
            }
            launch_charge_vjp(st, p, nshift, R, X.get(), Lm.get(), dz.get(), dw.get(), dqb.get(), dorb.get(), gH, gS);
            GSC_HIP(hipStreamSynchronize(st));
            inner += s1.inner_iters + s2.inner_iters;
            sri += s1.shift_rhs_iters + s2.shift_rhs_iters;
            outer = std::max(outer, std::max(s1.outer_iters, s2.outer_iters));
        }
        if (mem != GSC_MEM_DEVICE) {
            GSC_HIP(hipMemcpyAsync(dHval, gH, nv * 8, hipMemcpyDeviceToHost, st));
            GSC_HIP(hipMemcpyAsync(dSval, gS, nv * 8, hipMemcpyDeviceToHost, st));
        }
        GSC_HIP(hipStreamSynchronize(st));
        if (stats) {
            stats->outer_iters = outer;
            stats->inner_iters = inner;
            stats->shift_rhs_iters = sri;
        }
        return conv ? GSC_OK : GSC_NOT_CONVERGED;
    });
}

gsc_status gsc_csc_create(gsc_ctx *ctx, const gsc_pair *pair, const gsc_ased_geom *geom, const double *hubbard_u,
                          gsc_csc **out) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr && geom != nullptr && out != nullptr,
                    "ctx/pair/geom/out must not be NULL");
        GSC_REQUIRE(hubbard_u != nullptr, "hubbard_u must not be NULL");
        GSC_REQUIRE(geom->n_atoms >= 1 && geom->pos && geom->orb_atom && geom->trans, "incomplete geometry");
        for (int64_t a = 0; a < geom->n_atoms; ++a)
            GSC_REQUIRE(hubbard_u[a] > 0.0 && std::isfinite(hubbard_u[a]), "hubbard_u must be positive");
        DeviceGuard g(ctx->c.device);
        auto h = std::make_unique<gsc_csc>();
        csc_build(h->c, ctx->c, pair->p, *geom, hubbard_u);
        *out = h.release();
        return GSC_OK;
    });
}

void gsc_csc_destroy(gsc_csc *csc) {
    if (csc == nullptr) return;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    const int dev = csc->c.device;
    if (prev != dev) (void)hipSetDevice(dev);
    delete csc;
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

gsc_status gsc_csc_potential(gsc_csc *csc, const double *dq, double *V, int mem) {
    return guarded([&] {
        GSC_REQUIRE(csc != nullptr && dq != nullptr && V != nullptr, "csc/dq/V must not be NULL");
        DeviceGuard g(csc->c.ctx->device);
        hipStream_t st = csc->c.ctx->stream;
        const size_t n = static_cast<size_t>(csc->c.n_atoms);
        if (mem == GSC_MEM_DEVICE) {
            csc_potential(csc->c, dq, V, st);
            GSC_HIP(hipStreamSynchronize(st));
            return GSC_OK;
        }
        DevBuf<double> d(n), v(n);
        GSC_HIP(hipMemcpyAsync(d.get(), dq, n * 8, hipMemcpyHostToDevice, st));
        csc_potential(csc->c, d.get(), v.get(), st);
        GSC_HIP(hipMemcpyAsync(V, v.get(), n * 8, hipMemcpyDeviceToHost, st));
        GSC_HIP(hipStreamSynchronize(st));
        return GSC_OK;
    });
}

gsc_status gsc_csc_hamiltonian(gsc_csc *csc, gsc_pair *pair, const double *H0, const double *dq, int mem) {
    return guarded([&] {
        GSC_REQUIRE(csc != nullptr && pair != nullptr && H0 != nullptr && dq != nullptr, "NULL argument");
        Pair &p = pair->p;
        GSC_REQUIRE(p.nnzb == csc->c.nnzb && p.B == csc->c.B, "the pair does not match the csc handle");
        DeviceGuard g(csc->c.ctx->device);
        hipStream_t st = csc->c.ctx->stream;
        const size_t n = static_cast<size_t>(csc->c.n_atoms), nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
        DevBuf<double> d, h0, v(n);
        const double *dd = dq, *hh = H0;
        if (mem != GSC_MEM_DEVICE) {
            d.alloc(n);
            h0.alloc(nv);
            GSC_HIP(hipMemcpyAsync(d.get(), dq, n * 8, hipMemcpyHostToDevice, st));
            GSC_HIP(hipMemcpyAsync(h0.get(), H0, nv * 8, hipMemcpyHostToDevice, st));
            dd = d.get();
            hh = h0.get();
        }
        csc_potential(csc->c, dd, v.get(), st);
        csc_hamiltonian(csc->c, p, hh, v.get(), st);
        GSC_HIP(hipStreamSynchronize(st));
        return GSC_OK;
    });
}

void gsc_scc_opts_default(gsc_scc_opts *o) {
    if (o == nullptr) return;
    o->beta = 0.2;
    o->history = 4;
    o->tol = 1e-8;
    o->max_iter = 100;
    o->neutral = 0;
}

gsc_status gsc_scc(gsc_ctx *ctx, gsc_csc *csc, gsc_pair *pair, int nshift, const double *z, const double *w,
                   const double *valence, const gsc_scc_opts *sopts, const gsc_opts *opts, double *dq, double *q_orb,
                   double *e_band, int *iters, double *residual, double *e_fermi) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && csc != nullptr && pair != nullptr, "ctx/csc/pair must not be NULL");
        gsc_scc_opts so;
        gsc_scc_opts_default(&so);
        if (sopts) so = *sopts;
        GSC_REQUIRE(so.beta > 0.0 && so.history >= 0 && so.history <= 16 && so.tol > 0.0 && so.max_iter >= 1 &&
                        (so.neutral == 0 || so.neutral == 1),
                    "invalid scc options");
        GSC_REQUIRE((w != nullptr || so.neutral) && valence != nullptr && dq != nullptr,
                    "w/valence/dq must not be NULL");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        o.carry = GSC_CARRY_PROJECTED;
        validate_opts(o);
        validate_shifts(nshift, z, o.seed_index);
        Pair &p = pair->p;
        Csc &c = csc->c;
        GSC_REQUIRE(p.nnzb == c.nnzb && p.B == c.B, "the pair does not match the csc handle");
        DeviceGuard g(ctx->c.device);
        hipStream_t st = ctx->c.stream;
        const int64_t na = c.n_atoms, N = p.n;
        const int m = so.history;
        const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
        DevBuf<double> H0(nv), din(na), dout(na), f(na), V(na), xnew(na), qorb(N), Z(na), mx(1);
        DevBuf<double> Xh(std::max<int64_t>(1, m * na)), Fh(std::max<int64_t>(1, m * na)), dots(m * m + m + 1),
            gdev(m + 1);
        GSC_HIP(hipMemcpyAsync(H0.get(), p.H.get(), nv * 8, hipMemcpyDeviceToDevice, st));
        GSC_HIP(hipMemcpyAsync(din.get(), dq, na * 8, hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(Z.get(), valence, na * 8, hipMemcpyHostToDevice, st));
        std::vector<int64_t> orbs(N);
        for (int64_t i = 0; i < N; ++i) orbs[i] = i;
        // neutral mode: the grid's real parts, the valence count and the
        // per-shift projections (S G_k)_aa kept for the weights chosen after
        std::vector<double> E(nshift), t(nshift), wk;
        double ne = 0.0, ef = z[2 * (nshift - 1)];
        for (int k = 0; k < nshift; ++k) E[k] = z[2 * k];
        DevBuf<c128> sg, dz;
        DevBuf<double> tdev, dw, de, deb;
        if (so.neutral) {
            for (int k = 1; k < nshift; ++k) GSC_REQUIRE(E[k] > E[k - 1], "neutral mode needs increasing Re z");
            for (int64_t a = 0; a < na; ++a) ne += valence[a];
            GSC_REQUIRE(ne > 0.0, "neutral mode needs a positive valence count");
            sg.alloc(static_cast<size_t>(nshift) * N);
            dz.alloc(nshift); tdev.alloc(nshift); dw.alloc(nshift); de.alloc(N); deb.alloc(1);
            GSC_HIP(hipMemcpyAsync(dz.get(), z, nshift * sizeof(c128), hipMemcpyHostToDevice, st));
        }
        int it = 0, stored = 0;
        double res = 0.0, eb = 0.0;
        for (it = 1; it <= so.max_iter; ++it) {
            csc_potential(c, din.get(), V.get(), st);
            csc_hamiltonian(c, p, H0.get(), V.get(), st);
            if (so.neutral) {
                const gsc_status s = sg_solve(ctx->c, p, nshift, z, static_cast<int>(N), orbs.data(), o, sg.get(),
                                              nullptr);
                if (s < 0) return s;
                k_sg_trace<<<nshift, 256, 0, st>>>(static_cast<int>(N), sg.get(), tdev.get());
                GSC_HIP(hipMemcpyAsync(t.data(), tdev.get(), nshift * 8, hipMemcpyDeviceToHost, st));
                GSC_HIP(hipStreamSynchronize(st));
                // E_F by bisection: the count grows with E_F (-Im Tr S G > 0)
                double lo = E.front(), hi = E.back();
                GSC_REQUIRE(electron_count(E, t, hi, wk) >= ne, "the shift grid does not hold the electrons");
                while (hi - lo > 1e-13 * std::max(1.0, std::fabs(lo) + std::fabs(hi))) {
                    const double mid = 0.5 * (lo + hi);
                    if (electron_count(E, t, mid, wk) < ne) lo = mid;
                    else hi = mid;
                }
                ef = 0.5 * (lo + hi);
                truncated_trapezoid(E, ef, wk);
                GSC_HIP(hipMemcpyAsync(dw.get(), wk.data(), nshift * 8, hipMemcpyHostToDevice, st));
                k_mulliken<<<div_up(N, 256), 256, 0, st>>>(nshift, static_cast<int>(N), sg.get(), N, 1, dz.get(),
                                                           dw.get(), qorb.get(), de.get());
                k_sum<<<1, 256, 0, st>>>(static_cast<int>(N), de.get(), deb.get());
                GSC_HIP(hipGetLastError());
                GSC_HIP(hipMemcpyAsync(&eb, deb.get(), 8, hipMemcpyDeviceToHost, st));
            } else {
                const gsc_status s = gsc_mulliken_band(ctx, pair, nshift, z, w, static_cast<int>(N), orbs.data(), &o,
                                                       qorb.get(), nullptr, &eb, GSC_MEM_DEVICE, nullptr);
                if (s < 0) return s;
            }
            csc_charges(c, qorb.get(), Z.get(), din.get(), dout.get(), f.get(), st);
            max_abs(na, f.get(), mx.get(), st);
            GSC_HIP(hipMemcpyAsync(&res, mx.get(), 8, hipMemcpyDeviceToHost, st));
            GSC_HIP(hipStreamSynchronize(st));
            GSC_REQUIRE(std::isfinite(res), "non-finite charges in the self-consistency loop");
            if (res <= so.tol) break;
            const int mh = std::min(stored, m);
            std::vector<double> gh(std::max(mh, 1), 0.0);
            if (mh > 0) {
                anderson_dots(na, mh, f.get(), Fh.get(), dots.get(), st);
                std::vector<double> hd(mh * mh + mh);
                GSC_HIP(hipMemcpyAsync(hd.data(), dots.get(), hd.size() * 8, hipMemcpyDeviceToHost, st));
                GSC_HIP(hipStreamSynchronize(st));
                // normal equations of min |f - dF g| (mh <= 16), Gaussian elimination with pivoting
                std::vector<double> A(hd.begin(), hd.begin() + mh * mh), rhs(hd.begin() + mh * mh, hd.end());
                double tr = 0.0;
                for (int i = 0; i < mh; ++i) tr += A[i * mh + i];
                for (int i = 0; i < mh; ++i) A[i * mh + i] += 1e-14 * tr + 1e-300;
                for (int col = 0; col < mh; ++col) {
                    int piv = col;
                    for (int r = col + 1; r < mh; ++r)
                        if (std::fabs(A[r * mh + col]) > std::fabs(A[piv * mh + col])) piv = r;
                    for (int k = 0; k < mh; ++k) std::swap(A[col * mh + k], A[piv * mh + k]);
                    std::swap(rhs[col], rhs[piv]);
                    for (int r = col + 1; r < mh; ++r) {
                        const double fct = A[r * mh + col] / A[col * mh + col];
                        for (int k = col; k < mh; ++k) A[r * mh + k] -= fct * A[col * mh + k];
                        rhs[r] -= fct * rhs[col];
                    }
                }
                for (int r = mh - 1; r >= 0; --r) {
                    double v = rhs[r];
                    for (int k = r + 1; k < mh; ++k) v -= A[r * mh + k] * gh[k];
                    gh[r] = v / A[r * mh + r];
                }
                GSC_HIP(hipMemcpyAsync(gdev.get(), gh.data(), mh * 8, hipMemcpyHostToDevice, st));
            }
            anderson_mix(na, mh, so.beta, gdev.get(), din.get(), f.get(), Xh.get(), Fh.get(), xnew.get(), st);
            if (m > 0) {
                const int slot = stored % m;
                GSC_HIP(hipMemcpyAsync(Xh.get() + static_cast<size_t>(slot) * na, din.get(), na * 8,
                                       hipMemcpyDeviceToDevice, st));
                GSC_HIP(hipMemcpyAsync(Fh.get() + static_cast<size_t>(slot) * na, f.get(), na * 8,
                                       hipMemcpyDeviceToDevice, st));
                ++stored;
            }
            GSC_HIP(hipMemcpyAsync(din.get(), xnew.get(), na * 8, hipMemcpyDeviceToDevice, st));
        }
        const bool conv = it <= so.max_iter;
        if (!conv) {
            // the pair holds H0 + H^CSC of the last input charges
            csc_potential(c, din.get(), V.get(), st);
            csc_hamiltonian(c, p, H0.get(), V.get(), st);
        }
        GSC_HIP(hipMemcpyAsync(dq, din.get(), na * 8, hipMemcpyDeviceToHost, st));
        if (q_orb) GSC_HIP(hipMemcpyAsync(q_orb, qorb.get(), N * 8, hipMemcpyDeviceToHost, st));
        GSC_HIP(hipStreamSynchronize(st));
        if (e_band) *e_band = eb;
        if (iters) *iters = conv ? it : so.max_iter;
        if (residual) *residual = res;
        if (e_fermi) *e_fermi = ef;
        return conv ? GSC_OK : GSC_NOT_CONVERGED;
    });
}

gsc_status gsc_mulliken_band(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, const double *w,
                             int norb, const int64_t *orb_idx, const gsc_opts *opts, double *q_orb,
                             double *e_orb, double *e_band, int out_mem, gsc_stats *stats) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        validate_opts(o);
        validate_shifts(nshift, z, o.seed_index);
        GSC_REQUIRE(w != nullptr, "weights must not be NULL");
        GSC_REQUIRE(norb >= 1 && orb_idx != nullptr, "need at least one orbital");
        const Pair &p = pair->p;
        for (int r = 0; r < norb; ++r) GSC_REQUIRE(orb_idx[r] >= 0 && orb_idx[r] < p.n, "orbital index out of range");
        DeviceGuard g(ctx->c.device);
        hipStream_t st = ctx->c.stream;
        DevBuf<c128> sg(static_cast<size_t>(nshift) * norb);
        const gsc_status s = sg_solve(ctx->c, p, nshift, z, norb, orb_idx, o, sg.get(), stats);
        DevBuf<c128> dz(nshift);
        DevBuf<double> dw(nshift), dq(norb), de(norb), deb(1);
        GSC_HIP(hipMemcpyAsync(dz.get(), z, nshift * sizeof(c128), hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(dw.get(), w, nshift * sizeof(double), hipMemcpyHostToDevice, st));
        k_mulliken<<<div_up(norb, 256), 256, 0, st>>>(nshift, norb, sg.get(), norb, 1, dz.get(), dw.get(), dq.get(),
                                                      de.get());
        k_sum<<<1, 256, 0, st>>>(norb, de.get(), deb.get());
        GSC_HIP(hipGetLastError());
        const hipMemcpyKind kind = out_mem == GSC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (q_orb) GSC_HIP(hipMemcpyAsync(q_orb, dq.get(), norb * 8, kind, st));
        if (e_orb) GSC_HIP(hipMemcpyAsync(e_orb, de.get(), norb * 8, kind, st));
        double eb = 0.0;
        GSC_HIP(hipMemcpyAsync(&eb, deb.get(), 8, hipMemcpyDeviceToHost, st));
        GSC_HIP(hipStreamSynchronize(st));
        if (e_band) *e_band = eb;
        return s;
    });
}

gsc_status gsc_band_energy_vjp(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, const double *w,
                               int norb, const int64_t *orb_idx, double grad_E, const gsc_opts *opts, double *dHval,
                               double *dSval, double *e_band, int mem, gsc_stats *stats) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && pair != nullptr, "ctx/pair must not be NULL");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        validate_opts(o);
        validate_shifts(nshift, z, o.seed_index);
        GSC_REQUIRE(w != nullptr, "weights must not be NULL");
        GSC_REQUIRE(dHval != nullptr && dSval != nullptr, "dHval/dSval must not be NULL");
        GSC_REQUIRE(std::isfinite(grad_E), "grad_E must be finite");
        const Pair &p = pair->p;
        DeviceGuard g(ctx->c.device);
        hipStream_t st = ctx->c.stream;
        const int64_t N = p.n;
        const int B = p.B;
        // the columns this call covers
        std::vector<int64_t> cols;
        if (orb_idx == nullptr) {
            GSC_REQUIRE(norb == N, "orb_idx == NULL needs norb == N (every orbital)");
            cols.resize(N);
            for (int64_t c = 0; c < N; ++c) cols[c] = c;
        } else {
            GSC_REQUIRE(norb >= 1, "norb must be >= 1");
            std::vector<unsigned char> seen(N, 0);
            cols.assign(orb_idx, orb_idx + norb);
            for (const int64_t c : cols) {
                GSC_REQUIRE(c >= 0 && c < N, "orbital index out of range");
                GSC_REQUIRE(!seen[c], "orbital listed twice");
                seen[c] = 1;
            }
        }
        const int64_t R = static_cast<int64_t>(cols.size());
        o.carry = GSC_CARRY_PROJECTED;
        // projections of column c: every row b with a stored (b, c) entry,
        // i.e. the orbitals of the column blocks of c's block row (symmetric
        // pattern); the stored entry (b, c) sits in the mirror block
        int max_len = 0;
        for (int64_t I = 0; I < p.nb; ++I)
            max_len = std::max<int>(max_len, static_cast<int>(p.h_rowptr[I + 1] - p.h_rowptr[I]));
        const int Mu = max_len * B;
        GSC_REQUIRE(Mu + 1 <= 1024, "too many stored entries per column for the projected backward");
        std::vector<int32_t> mirror(p.nnzb);
        GSC_HIP(hipMemcpy(mirror.data(), p.mirror.get(), p.nnzb * 4, hipMemcpyDeviceToHost));
        ProjSpec ps;
        ps.M = Mu;
        ps.srow = true;
        ps.idx.assign(static_cast<size_t>(R) * Mu, 0);
        const int M = Mu + 1;
        std::vector<int64_t> vidx(static_cast<size_t>(R) * M, -1);
        for (int64_t r = 0; r < R; ++r) {
            const int64_t c = cols[r];
            const int64_t I = c / B, a = c % B;
            int m = 0;
            for (int64_t blk = p.h_rowptr[I]; blk < p.h_rowptr[I + 1]; ++blk) {
                const int64_t J = p.h_colidx[blk], mb = mirror[blk];
                for (int be = 0; be < B; ++be, ++m) {
                    ps.idx[static_cast<size_t>(r) * Mu + m] = static_cast<int32_t>(J * B + be);
                    vidx[static_cast<size_t>(r) * M + m] = (mb * B + be) * B + a;
                }
            }
            for (; m < Mu; ++m) ps.idx[static_cast<size_t>(r) * Mu + m] = static_cast<int32_t>(c);
        }
        const std::vector<int64_t> &rhs = cols;
        std::vector<double> wE(nshift);
        for (int k = 0; k < nshift; ++k) wE[k] = w[k] * z[2 * k];
        DevBuf<double> dwE(nshift);
        GSC_HIP(hipMemcpyAsync(dwE.get(), wE.data(), nshift * 8, hipMemcpyHostToDevice, st));
        DevBuf<c128> acc(static_cast<size_t>(R) * M * 3);
        GSC_HIP(hipMemsetAsync(acc.get(), 0, acc.n * sizeof(c128), st));
        SolveRequest req;
        req.pair = &p;
        req.K = nshift;
        req.z = z;
        req.R = static_cast<int>(R);
        req.rhs_idx = rhs.data();
        req.opts = o;
        req.out_mem = GSC_MEM_DEVICE;
        req.stats = stats;
        req.proj = &ps;
        req.vjp = true;
        req.wE = dwE.get();
        req.vjp_acc = acc.get();
        const gsc_status s = run_solve(ctx->c, req);
        // assemble into device buffers, then copy per mem
        const size_t nv = static_cast<size_t>(p.nnzb) * B * B;
        DevBuf<double> tH, tS;
        double *pH = dHval, *pS = dSval;
        if (mem != GSC_MEM_DEVICE) {
            tH.alloc(nv);
            tS.alloc(nv);
            GSC_HIP(hipMemcpyAsync(tH.get(), dHval, nv * 8, hipMemcpyHostToDevice, st));
            GSC_HIP(hipMemcpyAsync(tS.get(), dSval, nv * 8, hipMemcpyHostToDevice, st));
            pH = tH.get();
            pS = tS.get();
        }
        DevBuf<int64_t> dv(vidx.size());
        DevBuf<double> ecol(R), eb(1);
        GSC_HIP(hipMemcpyAsync(dv.get(), vidx.data(), vidx.size() * 8, hipMemcpyHostToDevice, st));
        const int64_t tot = R * M;
        k_vjp_assemble<<<div_up(tot, 256), 256, 0, st>>>(static_cast<int>(R), M, acc.get(), dv.get(), grad_E, pH, pS,
                                                         ecol.get());
        k_sum<<<1, 256, 0, st>>>(static_cast<int>(R), ecol.get(), eb.get());
        GSC_HIP(hipGetLastError());
        if (mem != GSC_MEM_DEVICE) {
            GSC_HIP(hipMemcpyAsync(dHval, tH.get(), nv * 8, hipMemcpyDeviceToHost, st));
            GSC_HIP(hipMemcpyAsync(dSval, tS.get(), nv * 8, hipMemcpyDeviceToHost, st));
        }
        double ebh = 0.0;
        GSC_HIP(hipMemcpyAsync(&ebh, eb.get(), 8, hipMemcpyDeviceToHost, st));
        GSC_HIP(hipStreamSynchronize(st));
        if (e_band) *e_band = ebh;
        return s;
    });
}

gsc_status gsc_profile_enable(gsc_ctx *ctx, int on) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr, "ctx must not be NULL");
        DeviceGuard g(ctx->c.device);
        GSC_HIP(hipStreamSynchronize(ctx->c.stream));
        ctx->c.prof.reset();
        ctx->c.prof.on = on != 0;
        ctx->c.prof.only = -1;
        return GSC_OK;
    });
}

gsc_status gsc_profile_select(gsc_ctx *ctx, const char *kernel) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr, "ctx must not be NULL");
        if (kernel == nullptr) { ctx->c.prof.only = -1; return GSC_OK; }
        for (int i = 0; i < KP_COUNT; ++i)
            if (std::strcmp(kernel, kernel_name(i)) == 0) { ctx->c.prof.only = i; return GSC_OK; }
        throw Error(GSC_E_ARG, std::string("unknown kernel name: ") + kernel);
    });
}

gsc_status gsc_profile_read(gsc_ctx *ctx, const char *kernel, double *total_ms, long long *launches,
                            double *bytes) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && kernel != nullptr, "ctx/kernel must not be NULL");
        {
            DeviceGuard g(ctx->c.device);
            GSC_HIP(hipStreamSynchronize(ctx->c.stream));
            ctx->c.prof.resolve();
        }
        for (int i = 0; i < KP_COUNT; ++i) {
            if (std::strcmp(kernel, kernel_name(i)) == 0) {
                const auto &a = ctx->c.prof.acc[i];
                if (total_ms) *total_ms = a.ms;
                if (launches) *launches = a.launches;
                if (bytes) *bytes = a.bytes;
                return GSC_OK;
            }
        }
        throw Error(GSC_E_ARG, std::string("unknown kernel name: ") + kernel);
    });
}

__global__ void k_extract_slot(int64_t n, int M, int slot, const c128 *in, c128 *out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) out[t] = in[t * M + slot];
}

gsc_status gsc_solve_batched(gsc_ctx *ctx, int nsys, const gsc_problem *problems, const gsc_opts *opts) {
    return guarded([&] {
        GSC_REQUIRE(ctx != nullptr && problems != nullptr && nsys >= 1, "bad batched arguments");
        gsc_opts o;
        gsc_opts_default(&o);
        if (opts) o = *opts;
        validate_opts(o);
        GSC_REQUIRE(o.graph_iters >= 0, "graph_iters must be >= 0");
        GSC_REQUIRE(o.batch_streams >= 0 && o.batch_streams <= 64, "batch_streams must be 0 .. 64");
        o.carry = GSC_CARRY_PROJECTED;
        const int graph_iters = o.graph_iters > 0 ? o.graph_iters : 4;
        DeviceGuard g(ctx->c.device);
        hipStream_t st = ctx->c.stream;
        std::vector<ProjSpec> specs(nsys);
        std::vector<SolveRequest> reqs(nsys);
        std::vector<DevBuf<c128>> outs(nsys);
        for (int i = 0; i < nsys; ++i) {
            const gsc_problem &pb = problems[i];
            GSC_REQUIRE(pb.pair != nullptr, "problem pair must not be NULL");
            validate_shifts(pb.nshift, pb.z, o.seed_index);
            GSC_REQUIRE(pb.nrhs >= 1 && pb.rhs_idx != nullptr, "each problem needs unit right-hand sides");
            const Pair &p = pb.pair->p;
            for (int r = 0; r < pb.nrhs; ++r)
                GSC_REQUIRE(pb.rhs_idx[r] >= 0 && pb.rhs_idx[r] < p.n, "rhs index out of range");
            specs[i].M = 1;
            specs[i].srow = true;
            specs[i].idx.resize(pb.nrhs);
            for (int r = 0; r < pb.nrhs; ++r) specs[i].idx[r] = static_cast<int32_t>(pb.rhs_idx[r]);
            outs[i].alloc(static_cast<size_t>(pb.nshift) * pb.nrhs * 2);
            SolveRequest &rq = reqs[i];
            rq.pair = &p;
            rq.K = pb.nshift;
            rq.z = pb.z;
            rq.R = pb.nrhs;
            rq.rhs_idx = pb.rhs_idx;
            rq.opts = o;
            rq.out_mem = GSC_MEM_DEVICE;
            rq.proj = &specs[i];
            rq.proj_out = outs[i].get();
            rq.stats = pb.stats;
            if (pb.stats) {
                pb.stats->inner_iters = 0;
                pb.stats->shift_rhs_iters = 0;
                pb.stats->switches = 0;
                pb.stats->restarts = 0;
                pb.stats->alg_bytes = 0.0;
                pb.stats->alg_bytes_inner = 0.0;
            }
        }
        hipEvent_t e0, e1;
        GSC_HIP(hipEventCreate(&e0));
        GSC_HIP(hipEventCreate(&e1));
        GSC_HIP(hipDeviceSynchronize());
        GSC_HIP(hipEventRecord(e0, st));
        std::vector<int> iters;
        const gsc_status s = run_batched(ctx->c, reqs, graph_iters, o.batch_streams > 0 ? o.batch_streams : 8,
                                         iters);
        GSC_HIP(hipDeviceSynchronize());
        GSC_HIP(hipEventRecord(e1, st));
        GSC_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        GSC_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (int i = 0; i < nsys; ++i) {
            const gsc_problem &pb = problems[i];
            const int64_t n = static_cast<int64_t>(pb.nshift) * pb.nrhs;
            if (pb.g_diag)
                k_extract_slot<<<div_up(n, 256), 256, 0, st>>>(n, 2, 0, outs[i].get(), reinterpret_cast<c128 *>(pb.g_diag));
            if (pb.w && (pb.q_orb || pb.e_orb)) {
                DevBuf<c128> dz(pb.nshift);
                DevBuf<double> dw(pb.nshift), dq(pb.nrhs), de(pb.nrhs);
                GSC_HIP(hipMemcpyAsync(dz.get(), pb.z, pb.nshift * sizeof(c128), hipMemcpyHostToDevice, st));
                GSC_HIP(hipMemcpyAsync(dw.get(), pb.w, pb.nshift * sizeof(double), hipMemcpyHostToDevice, st));
                k_mulliken<<<div_up(pb.nrhs, 256), 256, 0, st>>>(pb.nshift, pb.nrhs, outs[i].get() + 1,
                                                                 static_cast<size_t>(pb.nrhs) * 2, 2, dz.get(),
                                                                 dw.get(), pb.q_orb ? pb.q_orb : dq.get(),
                                                                 pb.e_orb ? pb.e_orb : de.get());
                GSC_HIP(hipStreamSynchronize(st));
            }
            if (pb.stats) pb.stats->seconds = ms * 1e-3;
        }
        GSC_HIP(hipGetLastError());
        GSC_HIP(hipStreamSynchronize(st));
        return s;
    });
}

}  // extern "C"
