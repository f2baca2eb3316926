// The H, S pair on the device, the ASED builder of eq. Hap-1 (Sec. 2.2) and
// its position derivative.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "pair.h"

namespace gsc {

// ------------------------------------------------------------------ pattern
void validate_and_upload(Pair &p, int block, int64_t nbrows, const int64_t *rowptr, const int32_t *colidx) {
    GSC_REQUIRE(block == 4 || block == 6, "block size must be 4 or 6");
    GSC_REQUIRE(nbrows > 0, "nbrows must be positive");
    GSC_REQUIRE(rowptr != nullptr && colidx != nullptr, "rowptr/colidx must not be NULL");
    GSC_REQUIRE(rowptr[0] == 0, "rowptr[0] must be 0");
    const int64_t nnzb = rowptr[nbrows];
    GSC_REQUIRE(nnzb > 0 && nnzb < (int64_t(1) << 31), "nnzb out of range");
    GSC_REQUIRE(nbrows * block < (int64_t(1) << 31), "N out of range");
    p.B = block;
    p.nb = nbrows;
    p.n = nbrows * block;
    p.nnzb = nnzb;
    p.h_rowptr.assign(rowptr, rowptr + nbrows + 1);
    p.h_colidx.assign(colidx, colidx + nnzb);
    for (int64_t i = 0; i < nbrows; ++i) {
        GSC_REQUIRE(rowptr[i + 1] >= rowptr[i], "rowptr must be non-decreasing");
        bool diag = false;
        for (int64_t b = rowptr[i]; b < rowptr[i + 1]; ++b) {
            GSC_REQUIRE(colidx[b] >= 0 && colidx[b] < nbrows, "column index out of range");
            if (b > rowptr[i]) GSC_REQUIRE(colidx[b] > colidx[b - 1], "column indices must be sorted and unique");
            diag |= colidx[b] == i;
        }
        GSC_REQUIRE(diag, "every diagonal block must be stored");
    }
    // mirror block (J, I) of every stored (I, J); the pattern must be symmetric
    std::vector<int32_t> brow(nnzb), mirror(nnzb);
    for (int64_t i = 0; i < nbrows; ++i)
        for (int64_t b = rowptr[i]; b < rowptr[i + 1]; ++b) brow[b] = static_cast<int32_t>(i);
    for (int64_t b = 0; b < nnzb; ++b) {
        const int32_t I = brow[b], J = colidx[b];
        const int32_t *lo = colidx + rowptr[J], *hi = colidx + rowptr[J + 1];
        const int32_t *f = std::lower_bound(lo, hi, I);
        GSC_REQUIRE(f != hi && *f == I, "pattern must be structurally symmetric");
        mirror[b] = static_cast<int32_t>(f - colidx);
    }
    std::vector<int32_t> rp32(nbrows + 1);
    for (int64_t i = 0; i <= nbrows; ++i) rp32[i] = static_cast<int32_t>(rowptr[i]);
    hipStream_t st = p.ctx->stream;
    p.rowptr.alloc(nbrows + 1);
    p.colidx.alloc(nnzb);
    p.brow.alloc(nnzb);
    p.mirror.alloc(nnzb);
    GSC_HIP(hipMemcpyAsync(p.rowptr.get(), rp32.data(), rp32.size() * 4, hipMemcpyHostToDevice, st));
    GSC_HIP(hipMemcpyAsync(p.colidx.get(), colidx, nnzb * 4, hipMemcpyHostToDevice, st));
    GSC_HIP(hipMemcpyAsync(p.brow.get(), brow.data(), nnzb * 4, hipMemcpyHostToDevice, st));
    GSC_HIP(hipMemcpyAsync(p.mirror.get(), mirror.data(), nnzb * 4, hipMemcpyHostToDevice, st));
    const size_t nv = static_cast<size_t>(nnzb) * block * block;
    p.H.alloc(nv);
    p.S.alloc(nv);
    GSC_HIP(hipStreamSynchronize(st));
}

void set_values(Pair &p, const double *H, const double *S, int mem) {
    const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
    const hipMemcpyKind kind = mem == GSC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipStream_t st = p.ctx->stream;
    if (H) GSC_HIP(hipMemcpyAsync(p.H.get(), H, nv * 8, kind, st));
    if (S) GSC_HIP(hipMemcpyAsync(p.S.get(), S, nv * 8, kind, st));
    GSC_HIP(hipStreamSynchronize(st));
    p.f32_valid = false;
}

__global__ void k_to_f32(size_t n, const double *a, float *b) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = static_cast<float>(a[i]);
}

void ensure_f32(Pair &p) {
    if (p.f32_valid) return;
    const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
    if (p.H32.n != nv) { p.H32.alloc(nv); p.S32.alloc(nv); }
    k_to_f32<<<div_up(static_cast<int64_t>(nv), 256), 256, 0, p.ctx->stream>>>(nv, p.H.get(), p.H32.get());
    k_to_f32<<<div_up(static_cast<int64_t>(nv), 256), 256, 0, p.ctx->stream>>>(nv, p.S.get(), p.S32.get());
    GSC_HIP(hipGetLastError());
    p.f32_valid = true;
}

// ------------------------------------------------------------------ ASED
struct AsedDev {
    const double *pos, *eps, *trans, *ang;
    const int32_t *orb_atom;
    double s0, r0, lam, kappa, theta;
};

// Geometry of entry (b, a, c): displacement d and distance r of the orbital
// centres; returns false when both orbitals sit on one atom.
__device__ inline bool entry_geom(const AsedDev &g, int B, int I, int J, int b, int a, int c, double d[3],
                                  double &r) {
    const int u = g.orb_atom[I * B + a], v = g.orb_atom[J * B + c];
    const double *t = g.trans + 3 * static_cast<size_t>(b);
    if (u == v && t[0] == 0.0 && t[1] == 0.0 && t[2] == 0.0) return false;
    for (int x = 0; x < 3; ++x) d[x] = g.pos[3 * static_cast<size_t>(v) + x] + t[x] - g.pos[3 * static_cast<size_t>(u) + x];
    r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    return true;
}

// unscaled off-site overlap s(r) * angular into S (temporary)
__global__ void k_ased_soff(int64_t nnzb, int B, const int32_t *brow, const int32_t *colidx, AsedDev g,
                            double *Soff) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t BB = static_cast<int64_t>(B) * B;
    if (t >= nnzb * BB) return;
    const int b = static_cast<int>(t / BB), e = static_cast<int>(t % BB);
    const int a = e / B, c = e % B;
    double d[3], r;
    double s = 0.0;
    if (entry_geom(g, B, brow[b], colidx[b], b, a, c, d, r))
        s = g.s0 * exp(-(r - g.r0) / g.lam) * g.ang[t];
    Soff[t] = s;
}

// per orbital row: sum of |S_off|
__global__ void k_ased_rowsum(int64_t n, int B, const int32_t *rowptr, const double *Soff, double *rowsum) {
    const int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int I = static_cast<int>(o / B), a = static_cast<int>(o % B);
    double s = 0.0;
    for (int b = rowptr[I]; b < rowptr[I + 1]; ++b)
        for (int c = 0; c < B; ++c) s += fabs(Soff[(static_cast<size_t>(b) * B + a) * B + c]);
    rowsum[o] = s;
}

__global__ void k_max_scale(int64_t n, const double *rowsum, double theta, double *scale) {
    __shared__ double lds[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, rowsum[i]);
    lds[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *scale = theta / lds[0];
}

__global__ void k_ased_final(int64_t nnzb, int B, const int32_t *brow, const int32_t *colidx, AsedDev g,
                             const double *scale, double *S, double *H) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t BB = static_cast<int64_t>(B) * B;
    if (t >= nnzb * BB) return;
    const int b = static_cast<int>(t / BB), e = static_cast<int>(t % BB);
    const int a = e / B, c = e % B;
    const int I = brow[b], J = colidx[b];
    const int o1 = I * B + a, o2 = J * B + c;
    const double c0 = *scale;
    double d[3], r;
    if (!entry_geom(g, B, I, J, b, a, c, d, r)) {
        const double diag = (o1 == o2) ? 1.0 : 0.0;
        S[t] = diag;
        H[t] = diag * g.eps[o1];
        return;
    }
    const double s = c0 * S[t];
    S[t] = s;
    H[t] = g.kappa * 0.5 * (g.eps[o1] + g.eps[o2]) * s;
}

// dE/dr / r summed with the mirror entry, times -d: contribution of every
// orbital row o1 to dE/dpos of its atom (deterministic, no atomics).
__global__ void k_ased_vjp_rows(int64_t n, int B, const int32_t *rowptr, const int32_t *colidx,
                                const int32_t *mirror, AsedDev g, double scale, const double *dH,
                                const double *dS, double *rowgrad) {
    const int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int I = static_cast<int>(o / B), a = static_cast<int>(o % B);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = rowptr[I]; b < rowptr[I + 1]; ++b) {
        const int J = colidx[b];
        const int mb = mirror[b];
        for (int c = 0; c < B; ++c) {
            double d[3], r;
            if (!entry_geom(g, B, I, J, b, a, c, d, r)) continue;
            const size_t e = (static_cast<size_t>(b) * B + a) * B + c;
            const size_t em = (static_cast<size_t>(mb) * B + c) * B + a;   // entry (o2, o1)
            const double kf = g.kappa * 0.5 * (g.eps[o] + g.eps[J * B + c]);
            const double gsum = (dS[e] + kf * dH[e]) + (dS[em] + kf * dH[em]);
            const double s = g.s0 * exp(-(r - g.r0) / g.lam) * g.ang[e];
            const double coef = gsum * scale * (-s / g.lam) / r;     // dE/dr / r (both entries)
            for (int x = 0; x < 3; ++x) acc[x] -= coef * d[x];        // d r / d pos_u = -d / r
        }
    }
    for (int x = 0; x < 3; ++x) rowgrad[3 * o + x] = acc[x];
}

__global__ void k_ased_vjp_atoms(int64_t n_atoms, const int32_t *aptr, const int32_t *aorb,
                                 const double *rowgrad, double *forces) {
    const int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (u >= n_atoms) return;
    double f[3] = {0.0, 0.0, 0.0};
    for (int j = aptr[u]; j < aptr[u + 1]; ++j)
        for (int x = 0; x < 3; ++x) f[x] -= rowgrad[3 * static_cast<size_t>(aorb[j]) + x];
    for (int x = 0; x < 3; ++x) forces[3 * u + x] = f[x];
}

namespace {
struct AsedUpload {
    DevBuf<double> pos, eps, trans, ang;
    DevBuf<int32_t> orb_atom;
    AsedDev dev{};
    AsedUpload(const Pair &p, const gsc_ased_geom *g) {
        GSC_REQUIRE(g != nullptr && g->pos && g->orb_atom && g->eps && g->trans && g->ang,
                    "ASED geometry arrays must not be NULL");
        GSC_REQUIRE(g->n_atoms > 0, "n_atoms must be positive");
        GSC_REQUIRE(g->lam > 0, "lam must be positive");
        for (int64_t o = 0; o < p.n; ++o)
            GSC_REQUIRE(g->orb_atom[o] >= 0 && g->orb_atom[o] < g->n_atoms, "orb_atom out of range");
        hipStream_t st = p.ctx->stream;
        const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
        pos.alloc(3 * g->n_atoms);
        eps.alloc(p.n);
        trans.alloc(3 * p.nnzb);
        ang.alloc(nv);
        orb_atom.alloc(p.n);
        GSC_HIP(hipMemcpyAsync(pos.get(), g->pos, 3 * g->n_atoms * 8, hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(eps.get(), g->eps, p.n * 8, hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(trans.get(), g->trans, 3 * p.nnzb * 8, hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(ang.get(), g->ang, nv * 8, hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(orb_atom.get(), g->orb_atom, p.n * 4, hipMemcpyHostToDevice, st));
        dev = AsedDev{pos.get(), eps.get(), trans.get(), ang.get(), orb_atom.get(),
                      g->s0, g->r0, g->lam, g->kappa, g->theta};
    }
};
}  // namespace

double ased_build(Pair &p, const gsc_ased_geom *g, double scale) {
    AsedUpload up(p, g);
    hipStream_t st = p.ctx->stream;
    const int64_t tot = p.nnzb * p.B * p.B;
    k_ased_soff<<<div_up(tot, 256), 256, 0, st>>>(p.nnzb, p.B, p.brow.get(), p.colidx.get(), up.dev, p.S.get());
    DevBuf<double> dscale(1);
    if (scale <= 0) {
        DevBuf<double> rowsum(p.n);
        k_ased_rowsum<<<div_up(p.n, 256), 256, 0, st>>>(p.n, p.B, p.rowptr.get(), p.S.get(), rowsum.get());
        k_max_scale<<<1, 256, 0, st>>>(p.n, rowsum.get(), g->theta, dscale.get());
        GSC_HIP(hipStreamSynchronize(st));
    } else {
        GSC_HIP(hipMemcpyAsync(dscale.get(), &scale, 8, hipMemcpyHostToDevice, st));
    }
    k_ased_final<<<div_up(tot, 256), 256, 0, st>>>(p.nnzb, p.B, p.brow.get(), p.colidx.get(), up.dev,
                                                   dscale.get(), p.S.get(), p.H.get());
    GSC_HIP(hipGetLastError());
    double c = 0.0;
    GSC_HIP(hipMemcpyAsync(&c, dscale.get(), 8, hipMemcpyDeviceToHost, st));
    GSC_HIP(hipStreamSynchronize(st));
    p.f32_valid = false;
    return c;
}

void ased_vjp(const Pair &p, const gsc_ased_geom *g, double scale, const double *dH, const double *dS, int mem,
              double *forces) {
    GSC_REQUIRE(scale > 0, "scale must be the positive constant used for the build");
    GSC_REQUIRE(forces != nullptr && dH != nullptr && dS != nullptr, "dH, dS, forces must not be NULL");
    AsedUpload up(p, g);
    hipStream_t st = p.ctx->stream;
    const size_t nv = static_cast<size_t>(p.nnzb) * p.B * p.B;
    DevBuf<double> ddH, ddS;
    const double *pH = dH, *pS = dS;
    if (mem != GSC_MEM_DEVICE) {
        ddH.alloc(nv);
        ddS.alloc(nv);
        GSC_HIP(hipMemcpyAsync(ddH.get(), dH, nv * 8, hipMemcpyHostToDevice, st));
        GSC_HIP(hipMemcpyAsync(ddS.get(), dS, nv * 8, hipMemcpyHostToDevice, st));
        pH = ddH.get();
        pS = ddS.get();
    }
    // atom -> orbital lists (host, deterministic order)
    std::vector<int32_t> aptr(g->n_atoms + 1, 0), aorb(p.n);
    for (int64_t o = 0; o < p.n; ++o) aptr[g->orb_atom[o] + 1]++;
    for (int64_t u = 0; u < g->n_atoms; ++u) aptr[u + 1] += aptr[u];
    std::vector<int32_t> fill(aptr.begin(), aptr.end() - 1);
    for (int64_t o = 0; o < p.n; ++o) aorb[fill[g->orb_atom[o]]++] = static_cast<int32_t>(o);
    DevBuf<int32_t> daptr(aptr.size()), daorb(aorb.size());
    GSC_HIP(hipMemcpyAsync(daptr.get(), aptr.data(), aptr.size() * 4, hipMemcpyHostToDevice, st));
    GSC_HIP(hipMemcpyAsync(daorb.get(), aorb.data(), aorb.size() * 4, hipMemcpyHostToDevice, st));
    DevBuf<double> rowgrad(3 * p.n), dforces(3 * g->n_atoms);
    k_ased_vjp_rows<<<div_up(p.n, 256), 256, 0, st>>>(p.n, p.B, p.rowptr.get(), p.colidx.get(), p.mirror.get(),
                                                      up.dev, scale, pH, pS, rowgrad.get());
    k_ased_vjp_atoms<<<div_up(g->n_atoms, 256), 256, 0, st>>>(g->n_atoms, daptr.get(), daorb.get(),
                                                             rowgrad.get(), dforces.get());
    GSC_HIP(hipGetLastError());
    GSC_HIP(hipMemcpyAsync(forces, dforces.get(), 3 * g->n_atoms * 8, hipMemcpyDeviceToHost, st));
    GSC_HIP(hipStreamSynchronize(st));
}

}  // namespace gsc
