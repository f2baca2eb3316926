// Charge-self-consistent term (Sec. 2.2, eq. Hap-CSC):
//   H^CSC_{ia,jb} = 1/2 S_{ia,jb} sum_k (gamma_ik + gamma_jk) dq_k
//                 = 1/2 S_{ia,jb} (V_i + V_j),   V = gamma dq,
// and the atom-level pieces of the self-consistency loop (charges, Anderson
// mixing).  gamma: U_i on the atom itself, else the Klopman-Ohno form
// e^2 / sqrt(r^2 + a^2), a = e^2 (1/U_i + 1/U_k) / 2, on the atom pairs the
// block pattern couples.  All arrays are small (atoms, stored entries).
#include <algorithm>
#include <array>
#include <vector>

#include "csc.h"

namespace gsc {

namespace {

constexpr double kE2 = 14.399645;  // e^2 / (4 pi eps0), eV * Angstrom

__global__ void k_csc_gamma(int64_t np, const int32_t *arow, const int32_t *acol, const int32_t *ablk,
                            const double *pos, const double *trans, const double *U, double *gamma) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= np) return;
    const int a = arow[t], k = acol[t];
    const double *tr = trans + 3 * static_cast<size_t>(ablk[t]);
    double d2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        const double d = pos[3 * static_cast<size_t>(k) + x] + tr[x] - pos[3 * static_cast<size_t>(a) + x];
        d2 += d * d;
    }
    if (a == k && d2 == 0.0) {
        gamma[t] = U[a];
    } else {
        const double h = 0.5 * kE2 * (1.0 / U[a] + 1.0 / U[k]);
        gamma[t] = kE2 / sqrt(d2 + h * h);
    }
}

__global__ void k_csc_potential(int64_t n, const int32_t *aptr, const int32_t *acol, const double *gamma,
                                const double *dq, double *V) {
    const int64_t a = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n) return;
    double v = 0.0;
    for (int32_t t = aptr[a]; t < aptr[a + 1]; ++t) v += gamma[t] * dq[acol[t]];
    V[a] = v;
}

__global__ void k_csc_values(int64_t nnzb, int B, const int32_t *brow, const int32_t *colidx,
                             const int32_t *orb_atom, const double *S, const double *H0, const double *V, double *H) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nnzb * B * B) return;
    const int64_t b = t / (B * B);
    const int e = static_cast<int>(t % (B * B)), a = e / B, c = e % B;
    const int u = orb_atom[static_cast<int64_t>(brow[b]) * B + a];
    const int v = orb_atom[static_cast<int64_t>(colidx[b]) * B + c];
    H[t] = H0[t] + 0.5 * S[t] * (V[u] + V[v]);
}

__global__ void k_csc_charges(int64_t n, const int32_t *optr, const int32_t *oidx, const double *q_orb,
                              const double *Z, const double *dq_in, double *dq_out, double *f) {
    const int64_t a = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n) return;
    double Q = 0.0;
    for (int32_t t = optr[a]; t < optr[a + 1]; ++t) Q += q_orb[oidx[t]];
    const double o = Q - Z[a];
    dq_out[a] = o;
    f[a] = o - dq_in[a];
}

__global__ __launch_bounds__(256) void k_max_abs(int64_t n, const double *x, double *out) {
    __shared__ double l[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(x[i]));
    l[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) l[threadIdx.x] = fmax(l[threadIdx.x], l[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = l[0];
}

// block d: dot (i, j) = (f - F_i).(f - F_j) for d < mh*mh, else (f - F_i).f
__global__ __launch_bounds__(256) void k_anderson_dots(int64_t n, int mh, const double *f, const double *Fh,
                                                       double *out) {
    __shared__ double l[256];
    const int d = blockIdx.x;
    const int i = d < mh * mh ? d / mh : d - mh * mh;
    const int j = d < mh * mh ? d % mh : -1;
    const double *Fi = Fh + static_cast<size_t>(i) * n;
    const double *Fj = j >= 0 ? Fh + static_cast<size_t>(j) * n : nullptr;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) {
        const double di = f[k] - Fi[k];
        s += di * (j >= 0 ? f[k] - Fj[k] : f[k]);
    }
    l[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) l[threadIdx.x] += l[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[d] = l[0];
}

__global__ void k_anderson_mix(int64_t n, int mh, double beta, const double *g, const double *x, const double *f,
                               const double *Xh, const double *Fh, double *xnew) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double v = x[k] + beta * f[k];
    for (int i = 0; i < mh; ++i) {
        const double dx = x[k] - Xh[static_cast<size_t>(i) * n + k];
        const double df = f[k] - Fh[static_cast<size_t>(i) * n + k];
        v -= g[i] * (dx + beta * df);
    }
    xnew[k] = v;
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

void csc_build(Csc &c, Ctx &ctx, const Pair &p, const gsc_ased_geom &g, const double *U) {
    c.ctx = &ctx;
    c.device = ctx.device;
    c.n_atoms = g.n_atoms;
    c.B = p.B;
    c.N = p.n;
    c.nnzb = p.nnzb;
    const int B = p.B;
    // atom pairs of every stored block, grouped by the first atom
    std::vector<std::vector<std::array<int32_t, 2>>> rows(static_cast<size_t>(g.n_atoms));
    for (int64_t I = 0; I < p.nb; ++I) {
        std::vector<int32_t> ai;
        for (int a = 0; a < B; ++a) ai.push_back(g.orb_atom[I * B + a]);
        std::sort(ai.begin(), ai.end());
        ai.erase(std::unique(ai.begin(), ai.end()), ai.end());
        for (int64_t b = p.h_rowptr[I]; b < p.h_rowptr[I + 1]; ++b) {
            const int64_t J = p.h_colidx[b];
            std::vector<int32_t> aj;
            for (int cc = 0; cc < B; ++cc) aj.push_back(g.orb_atom[J * B + cc]);
            std::sort(aj.begin(), aj.end());
            aj.erase(std::unique(aj.begin(), aj.end()), aj.end());
            for (int32_t a : ai)
                for (int32_t k : aj) rows[a].push_back({k, static_cast<int32_t>(b)});
        }
    }
    std::vector<int32_t> aptr(g.n_atoms + 1, 0), arow, acol, ablk;
    for (int64_t a = 0; a < g.n_atoms; ++a) {
        for (const auto &e : rows[a]) {
            arow.push_back(static_cast<int32_t>(a));
            acol.push_back(e[0]);
            ablk.push_back(e[1]);
        }
        aptr[a + 1] = static_cast<int32_t>(acol.size());
    }
    c.npairs = static_cast<int64_t>(acol.size());
    // atom -> orbitals
    std::vector<int32_t> optr(g.n_atoms + 1, 0), oidx(p.n);
    for (int64_t o = 0; o < p.n; ++o) {
        GSC_REQUIRE(g.orb_atom[o] >= 0 && g.orb_atom[o] < g.n_atoms, "orb_atom out of range");
        ++optr[g.orb_atom[o] + 1];
    }
    for (int64_t a = 0; a < g.n_atoms; ++a) optr[a + 1] += optr[a];
    std::vector<int32_t> fill(optr.begin(), optr.end() - 1);
    for (int64_t o = 0; o < p.n; ++o) oidx[fill[g.orb_atom[o]]++] = static_cast<int32_t>(o);
    hipStream_t st = ctx.stream;
    auto up_i = [&](DevBuf<int32_t> &d, const std::vector<int32_t> &h) {
        d.alloc(std::max<size_t>(h.size(), 1));
        if (!h.empty()) GSC_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    };
    auto up_d = [&](DevBuf<double> &d, const double *h, size_t n) {
        d.alloc(std::max<size_t>(n, 1));
        if (n) GSC_HIP(hipMemcpyAsync(d.get(), h, n * 8, hipMemcpyHostToDevice, st));
    };
    up_i(c.aptr, aptr);
    up_i(c.arow, arow);
    up_i(c.acol, acol);
    up_i(c.ablk, ablk);
    up_i(c.optr, optr);
    up_i(c.oidx, oidx);
    std::vector<int32_t> oa(g.orb_atom, g.orb_atom + p.n);
    up_i(c.orb_atom, oa);
    up_d(c.pos, g.pos, 3 * static_cast<size_t>(g.n_atoms));
    up_d(c.trans, g.trans, 3 * static_cast<size_t>(p.nnzb));
    up_d(c.U, U, static_cast<size_t>(g.n_atoms));
    c.gamma.alloc(std::max<int64_t>(c.npairs, 1));
    if (c.npairs > 0) {
        k_csc_gamma<<<blocks_for(c.npairs), 256, 0, st>>>(c.npairs, c.arow.get(), c.acol.get(), c.ablk.get(),
                                                          c.pos.get(), c.trans.get(), c.U.get(), c.gamma.get());
        GSC_HIP(hipGetLastError());
    }
    GSC_HIP(hipStreamSynchronize(st));
}

void csc_potential(const Csc &c, const double *dq, double *V, hipStream_t st) {
    k_csc_potential<<<blocks_for(c.n_atoms), 256, 0, st>>>(c.n_atoms, c.aptr.get(), c.acol.get(), c.gamma.get(), dq,
                                                           V);
    GSC_HIP(hipGetLastError());
}

void csc_hamiltonian(const Csc &c, Pair &p, const double *H0, const double *V, hipStream_t st) {
    const int64_t n = p.nnzb * p.B * p.B;
    k_csc_values<<<blocks_for(n), 256, 0, st>>>(p.nnzb, p.B, p.brow.get(), p.colidx.get(), c.orb_atom.get(),
                                                p.S.get(), H0, V, p.H.get());
    GSC_HIP(hipGetLastError());
    p.f32_valid = false;
}

void csc_charges(const Csc &c, const double *q_orb, const double *Z, const double *dq_in, double *dq_out, double *f,
                 hipStream_t st) {
    k_csc_charges<<<blocks_for(c.n_atoms), 256, 0, st>>>(c.n_atoms, c.optr.get(), c.oidx.get(), q_orb, Z, dq_in,
                                                         dq_out, f);
    GSC_HIP(hipGetLastError());
}

void max_abs(int64_t n, const double *x, double *out, hipStream_t st) {
    k_max_abs<<<1, 256, 0, st>>>(n, x, out);
    GSC_HIP(hipGetLastError());
}

void anderson_dots(int64_t n, int mh, const double *f, const double *Fh, double *out, hipStream_t st) {
    if (mh <= 0) return;
    k_anderson_dots<<<mh * mh + mh, 256, 0, st>>>(n, mh, f, Fh, out);
    GSC_HIP(hipGetLastError());
}

void anderson_mix(int64_t n, int mh, double beta, const double *g, const double *x, const double *f,
                  const double *Xh, const double *Fh, double *xnew, hipStream_t st) {
    k_anderson_mix<<<blocks_for(n), 256, 0, st>>>(n, mh, beta, g, x, f, Xh, Fh, xnew);
    GSC_HIP(hipGetLastError());
}

}  // namespace gsc
