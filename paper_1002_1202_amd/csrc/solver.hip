// Generalized shifted COCG (Sec. 3.3) for one tile of right-hand sides.
//
// Per outer iteration n (every kernel masks finished columns):
//   spmm_seed   q = A_s p = z_s S p - H p,  partial p^T q          (eq. CGp:r)
//   ctrl        alpha = rho / p^T q; per shift pi_{n+1} (eq. Shift:pi with the
//               derived sign) and the update coefficients 1/pi_n, beta^k, alpha^k
//   shift upd.  p^k <- r'_n/pi_n + beta^k p^k,  x^k <- x^k + alpha^k p^k
//               (full carry: deferred and applied m steps per pass; projected
//               carry: on the projections c^T x^k, c^T p^k)
//   update_r    r <- r - alpha q                                    (eq. CGp:r)
//   inner CG    r' = S^{-1} r (Sec. 3.3: S is positive definite and close to I)
//   post        rho' = r'^T r, beta = rho'/rho; pi shift; ||r||/(|pi| ||b||)
//               freezes converged shifts (eq. Collinear); seed switching
//   p_update    p <- r' + beta p                                    (eq. CGp:p)
// All scalar recurrences, dots and reductions are FP64; vectors and products
// are complex<T> (T = double, or float in the mixed mode).
#include <algorithm>
#include <array>
#include <chrono>
#include <memory>
#include <thread>
#include <cmath>
#include <cstring>

#include "solver.h"
#include "spmm.h"

namespace gsc {

// budget of the Chebyshev column blocks' streamed vectors (of the 256 MB
// infinity cache)
constexpr double kChebBlockBytes = 224.0e6;
constexpr int kBatchTile = 128;   // default rhs per job of gsc_solve_batched

// ------------------------------------------------------------------ helpers
template <typename V>
__device__ inline V block_sum(V v, V *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] = lds[threadIdx.x] + lds[threadIdx.x + s];
        __syncthreads();
    }
    V r = lds[0];
    __syncthreads();
    return r;
}

// Row range of the vector kernels: group g covers rows [g*Lr, (g+1)*Lr).
#define ELEM_LOOP_BEGIN                                     \
    int cx, g;                                              \
    xcd_remap(cx, g);                                       \
    const int lane = threadIdx.x & 63;                      \
    const int wv = wave_id();                               \
    const int col = cx * 64 + lane;                         \
    const int i0 = g * Lr;                                  \
    const int i1 = min(N, i0 + Lr);

template <typename V>
__device__ inline void wave_partial_store(V v, V *partial, int g, int Rp, int col) {
    __shared__ V red[kWavesPerBlock][64];
    const int lane = threadIdx.x & 63;
    red[threadIdx.x >> 6][lane] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        V s = red[0][lane];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) s = s + red[k][lane];
        partial[static_cast<size_t>(g) * Rp + col] = s;
    }
}

// ------------------------------------------------------------------ init
__global__ void k_init_cols(int R, int Rp, int seed0, ColState cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Rp) return;
    cs.seed[c] = seed0;
    cs.done[c] = c >= R ? 1 : 0;
    cs.alpha_prev[c] = {1.0, 0.0};
    cs.beta_prev[c] = {0.0, 0.0};
    cs.alpha[c] = {0.0, 0.0};
    cs.rho[c] = {0.0, 0.0};
    cs.flags[c] = 0;
    cs.applied[c] = 0;
    cs.sw[c] = 0;
    cs.shift_iters[c] = 0;
    cs.iters[c] = 0;
    cs.inner_total[c] = 0;
    cs.zres[c] = 0;
    cs.inner_done[c] = 1;
    cs.inner_count[c] = 0;
    cs.wres[c] = 1.0;
}

__global__ void k_init_shifts(int K, int R, int Rp, ShiftState ss) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(K) * Rp) return;
    const int c = static_cast<int>(t % Rp);
    ss.pi[t] = {1.0, 0.0};
    ss.pi_prev[t] = {1.0, 0.0};
    ss.pi_next[t] = {1.0, 0.0};
    ss.omega[t] = {1.0, 0.0};
    ss.res[t] = 0.0;
    ss.last[t] = c < R ? kFrozenNever : -1;
    if (ss.dpi != nullptr) {
        ss.dpi[t] = {0.0, 0.0};
        ss.dpi_prev[t] = {0.0, 0.0};
        ss.dpi_next[t] = {0.0, 0.0};
        ss.domega[t] = {0.0, 0.0};
    }
}

// r = b; res = d = r; partial ||r||^2.  Unit rhs (rhs != null) or dense B[c][i].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_rhs(int N, int Rp, int Lr, int R, const int64_t *rhs,
                                                     const c128 *Bd, cpx<T> *r, cpx<T> *res, cpx<T> *d,
                                                     double *partial) {
    ELEM_LOOP_BEGIN
    double acc = 0.0;
    const int64_t j = (rhs != nullptr && col < R) ? rhs[col] : -1;
    for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
        cpx<T> v{0, 0};
        if (col < R) {
            if (rhs != nullptr) v = (i == j) ? cpx<T>{1, 0} : cpx<T>{0, 0};
            else v = ccast<T>(Bd[static_cast<size_t>(col) * N + i]);
        }
        const size_t e = static_cast<size_t>(i) * Rp + col;
        r[e] = v;
        res[e] = v;
        d[e] = v;
        acc += static_cast<double>(v.re) * v.re + static_cast<double>(v.im) * v.im;
    }
    wave_partial_store(acc, partial, g, Rp, col);
}

template <typename T>
__global__ void k_zero_done_cols(int K, int R, int N, size_t ldk, const int *done, cpx<T> *X) {
    // x^k = 0 for every shift of a column that is done before its first
    // step (b = 0); every other column's x^k is written by its first pass
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int c = blockIdx.y; c < R; c += gridDim.y) {
        if (!done[c]) continue;
        for (int k = 0; k < K; ++k) X[static_cast<size_t>(k) * ldk + static_cast<size_t>(c) * N + i] = {0, 0};
    }
}

// ------------------------------------------------------------------ column kernels
// ||r||^2 reduction; prepares the inner solve of S r' = r.
__global__ __launch_bounds__(kBlock) void k_col_rnorm(int Rp, int G, const double *partial, int init,
                                                      double inner_tol, ColState cs) {
    __shared__ double lds[kBlock];
    const int c = blockIdx.x;
    double v = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) v += partial[static_cast<size_t>(g) * Rp + c];
    const double rn2 = block_sum(v, lds);
    if (threadIdx.x != 0) return;
    if (cs.done[c]) { cs.inner_done[c] = 1; return; }
    cs.rnorm2[c] = rn2;
    if (init) {
        cs.bnorm[c] = sqrt(rn2);
        if (rn2 == 0.0) cs.done[c] = 1;      // b = 0: x = 0 for every shift
    }
    if (!isfinite(rn2)) { cs.flags[c] |= FLAG_NAN; cs.done[c] = 1; }
    cs.rr[c] = rn2;
    cs.rr_stop[c] = inner_tol * inner_tol * rn2;
    cs.zres[c] = rn2 == 0.0 ? 1 : 0;
    cs.inner_done[c] = (rn2 == 0.0 || cs.done[c]) ? 1 : 0;
    cs.cg_first[c] = 1;
    cs.inner_count[c] = 0;
}

__global__ __launch_bounds__(kBlock) void k_cg_a(int Rp, int G, const double *partial, ColState cs) {
    __shared__ double lds[kBlock];
    const int c = blockIdx.x;
    if (cs.inner_done[c]) return;
    double v = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) v += partial[static_cast<size_t>(g) * Rp + c];
    const double dw = block_sum(v, lds);
    if (threadIdx.x != 0) return;
    if (!(dw > 0.0)) {
        cs.flags[c] |= isfinite(dw) ? FLAG_NOT_SPD : FLAG_NAN;
        cs.inner_done[c] = 1;
        cs.done[c] = 1;
        cs.cg_a[c] = 0.0;
        return;
    }
    cs.cg_a[c] = cs.rr[c] / dw;
    if (cs.cg_ha != nullptr && cs.inner_count[c] < kHist)
        cs.cg_ha[static_cast<size_t>(c) * kHist + cs.inner_count[c]] = cs.cg_a[c];
}

__global__ __launch_bounds__(kBlock) void k_cg_b(int Rp, int G, const double *partial, int inner_max,
                                                 ColState cs) {
    __shared__ double lds[kBlock];
    const int c = blockIdx.x;
    if (cs.inner_done[c]) return;
    double v = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) v += partial[static_cast<size_t>(g) * Rp + c];
    const double rr_new = block_sum(v, lds);
    if (threadIdx.x != 0) return;
    const double rr = cs.rr[c];
    cs.cg_b[c] = rr_new / rr;
    if (cs.cg_hb != nullptr && cs.inner_count[c] < kHist)
        cs.cg_hb[static_cast<size_t>(c) * kHist + cs.inner_count[c]] = cs.cg_b[c];
    cs.rr[c] = rr_new;
    cs.cg_first[c] = 0;
    cs.inner_total[c] += 1;
    const int cnt = ++cs.inner_count[c];
    if (!isfinite(rr_new)) {
        cs.flags[c] |= FLAG_NAN;
        cs.done[c] = 1;
        cs.inner_done[c] = 1;
    } else if (rr_new <= cs.rr_stop[c]) {
        cs.inner_done[c] = 1;
    } else if (cnt >= inner_max) {
        cs.flags[c] |= FLAG_INNER;
        cs.inner_done[c] = 1;
    }
}

// alpha = rho / (p^T A_s p) and the shift coefficients of step n (slot).
__global__ __launch_bounds__(kBlock) void k_ctrl(int K, int Rp, int G, int n, int slot, const c128 *partial,
                                                 ColState cs, ShiftState ss) {
    __shared__ c128 lds[kBlock];
    __shared__ c128 s_alpha, s_tail, s_zs;
    __shared__ int s_ok;
    __shared__ long long s_cnt[kBlock];
    const int c = blockIdx.x;
    if (cs.done[c]) return;
    c128 v{0, 0};
    for (int g = threadIdx.x; g < G; g += kBlock) v = v + partial[static_cast<size_t>(g) * Rp + c];
    const c128 mu = block_sum(v, lds);
    if (threadIdx.x == 0) {
        cs.sw[c] = 0;
        const c128 rho = cs.rho[c];
        const c128 alpha = cdiv(rho, mu);
        int ok = 1;
        if (!cfinite(mu) || !cfinite(alpha)) {
            cs.flags[c] |= cfinite(mu) ? FLAG_BREAKDOWN : FLAG_NAN;
            ok = 0;
        } else if (cabs(mu) == 0.0 || cabs(alpha) == 0.0) {
            cs.flags[c] |= FLAG_BREAKDOWN;
            ok = 0;
        }
        if (!ok) cs.done[c] = 1;
        cs.alpha[c] = alpha;
        s_alpha = alpha;
        s_tail = cdiv(alpha * cs.beta_prev[c], cs.alpha_prev[c]);
        s_zs = ss.z[cs.seed[c]];
        s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) return;
    const c128 alpha = s_alpha, tail = s_tail, zs = s_zs;
    long long cnt = 0;
    for (int k = threadIdx.x; k < K; k += kBlock) {
        const size_t idx = static_cast<size_t>(k) * Rp + c;
        if (ss.last[idx] != kFrozenNever) continue;
        ++cnt;
        const c128 pi = ss.pi[idx], pim = ss.pi_prev[idx];
        const c128 delta = ss.z[k] - zs;
        const c128 lead = c128{1.0, 0.0} + alpha * delta;
        const c128 pin = lead * pi + tail * (pi - pim);
        ss.pi_next[idx] = pin;
        const c128 q = cdiv(pim, pi);
        const c128 ak = cdiv(alpha * pi, pin);      // alpha^k_n
        ss.ra[coef_at(ss, k, c, slot)] = cdiv(c128{1.0, 0.0}, pi);
        ss.rb[coef_at(ss, k, c, slot)] = (q * q) * cs.beta_prev[c];
        ss.rc[coef_at(ss, k, c, slot)] = ss.omega[idx] * ak;
        if (ss.dpi != nullptr) {
            // d/dz_k of the recurrence at a fixed seed process (delta' = 1)
            const c128 dpi = ss.dpi[idx], dpim = ss.dpi_prev[idx];
            const c128 dpin = alpha * pi + lead * dpi + tail * (dpi - dpim);
            ss.dpi_next[idx] = dpin;
            const c128 dak = cdiv(alpha * (dpi * pin - pi * dpin), pin * pin);
            const c128 dbk = cdiv(2.0 * cs.beta_prev[c] * q * (dpim * pi - pim * dpi), pi * pi);
            ss.rda[coef_at(ss, k, c, slot)] = cdiv(c128{-dpi.re, -dpi.im}, pi * pi);
            ss.rdb[coef_at(ss, k, c, slot)] = dbk;
            ss.rdc[coef_at(ss, k, c, slot)] = ss.domega[idx] * ak + ss.omega[idx] * dak;
        }
    }
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) s_cnt[threadIdx.x] += s_cnt[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cs.shift_iters[c] += s_cnt[0];
        cs.iters[c] += 1;
        if (cs.act_hist != nullptr) {
            atomicAdd(reinterpret_cast<unsigned long long *>(cs.act_hist + n),
                      static_cast<unsigned long long>(s_cnt[0]));
            atomicAdd(reinterpret_cast<unsigned long long *>(cs.col_hist + n), 1ull);
        }
    }
}

// rho' = r'^T r; beta; pi shift; freeze; seed switch / collinear restart.
__global__ __launch_bounds__(kBlock) void k_post(int K, int Rp, int G, int n, int full_carry,
                                                 const c128 *partial, double tol, ColState cs,
                                                 ShiftState ss, c128 *proj_h, c128 *proj_dh, int M) {
    __shared__ c128 lds[kBlock];
    __shared__ double s_res[kBlock];
    __shared__ int s_k[kBlock];
    __shared__ int s_cnt[kBlock];
    __shared__ int s_sw;
    __shared__ c128 s_c, s_cm;
    const int c = blockIdx.x;
    if (cs.done[c]) return;
    c128 v{0, 0};
    for (int g = threadIdx.x; g < G; g += kBlock) v = v + partial[static_cast<size_t>(g) * Rp + c];
    const c128 rho_new = block_sum(v, lds);
    const double rn = sqrt(cs.rnorm2[c]);
    const double bn = cs.bnorm[c];
    double best = -1.0;
    int bestk = 0x7fffffff, cnt = 0;
    for (int k = threadIdx.x; k < K; k += kBlock) {
        const size_t idx = static_cast<size_t>(k) * Rp + c;
        if (ss.last[idx] != kFrozenNever) continue;
        const c128 pin = ss.pi_next[idx];
        ss.pi_prev[idx] = ss.pi[idx];
        ss.pi[idx] = pin;
        if (ss.dpi != nullptr) {
            ss.dpi_prev[idx] = ss.dpi[idx];
            ss.dpi[idx] = ss.dpi_next[idx];
        }
        const double res = cabs(ss.omega[idx]) * rn / (cabs(pin) * bn);
        ss.res[idx] = res;
        if (!(res > tol)) {
            ss.last[idx] = n;
        } else {
            ++cnt;
            if (res > best) { best = res; bestk = k; }
        }
    }
    s_res[threadIdx.x] = best;
    s_k[threadIdx.x] = bestk;
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double r2 = s_res[threadIdx.x + s];
            const int k2 = s_k[threadIdx.x + s];
            if (r2 > s_res[threadIdx.x] || (r2 == s_res[threadIdx.x] && k2 < s_k[threadIdx.x])) {
                s_res[threadIdx.x] = r2;
                s_k[threadIdx.x] = k2;
            }
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cs.wres[c] = s_res[0];
        const c128 rho = cs.rho[c];
        const c128 beta = cdiv(rho_new, rho);
        cs.alpha_prev[c] = cs.alpha[c];
        cs.beta_prev[c] = beta;
        cs.rho[c] = rho_new;
        int sw = 0;
        if (s_cnt[0] == 0) {
            cs.done[c] = 1;
        } else if (!cfinite(rho_new) || !cfinite(beta)) {
            cs.flags[c] |= FLAG_NAN;
            cs.done[c] = 1;
        } else if (cabs(rho_new) == 0.0) {
            cs.flags[c] |= FLAG_BREAKDOWN;
            cs.done[c] = 1;
        } else {
            const int seed = cs.seed[c];
            if (ss.last[static_cast<size_t>(seed) * Rp + c] != kFrozenNever) {
                const int sn = s_k[0];
                const size_t ix = static_cast<size_t>(sn) * Rp + c;
                const c128 cc = ss.pi[ix], ccm = ss.pi_prev[ix];
                if (full_carry) {
                    // exact seed switch: rescale the seed quantities by pi of
                    // the new seed; shifted iterates are invariant
                    const c128 q = cdiv(ccm, cc);
                    cs.rho[c] = cdiv(rho_new, cc * cc);
                    cs.beta_prev[c] = (q * q) * beta;
                    cs.alpha_prev[c] = cs.alpha[c] * q;
                    sw = 1;
                } else {
                    // collinear restart on the current residual
                    cs.alpha_prev[c] = {1.0, 0.0};
                    cs.beta_prev[c] = {0.0, 0.0};
                    sw = 2;
                }
                cs.seed[c] = sn;
                cs.swc[c] = cc;
                cs.swcm[c] = ccm;
                s_c = cc;
                s_cm = ccm;
            }
        }
        cs.sw[c] = sw;
        s_sw = cs.done[c] ? 0 : sw;
    }
    __syncthreads();
    const int sw = s_sw;
    if (sw == 1) {
        const c128 cc = s_c, ccm = s_cm;
        for (int k = threadIdx.x; k < K; k += kBlock) {
            const size_t idx = static_cast<size_t>(k) * Rp + c;
            ss.pi[idx] = cdiv(ss.pi[idx], cc);
            ss.pi_prev[idx] = cdiv(ss.pi_prev[idx], ccm);
            if (ss.dpi != nullptr) {
                ss.dpi[idx] = cdiv(ss.dpi[idx], cc);
                ss.dpi_prev[idx] = cdiv(ss.dpi_prev[idx], ccm);
            }
        }
    } else if (sw == 2) {
        for (int k = threadIdx.x; k < K; k += kBlock) {
            const size_t idx = static_cast<size_t>(k) * Rp + c;
            if (ss.last[idx] == kFrozenNever) {
                const c128 pik = ss.pi[idx];
                if (ss.dpi != nullptr)
                    // omega_k / pi_k(z): d/dz = domega/pi - omega dpi / pi^2
                    ss.domega[idx] = cdiv(ss.domega[idx], pik) - cdiv(ss.omega[idx] * ss.dpi[idx], pik * pik);
                ss.omega[idx] = cdiv(ss.omega[idx], pik);
            }
            ss.pi[idx] = {1.0, 0.0};
            ss.pi_prev[idx] = {1.0, 0.0};
            if (ss.dpi != nullptr) {
                ss.dpi[idx] = {0.0, 0.0};
                ss.dpi_prev[idx] = {0.0, 0.0};
            }
            if (proj_h != nullptr)
                for (int m = 0; m < M; ++m) {
                    proj_h[(static_cast<size_t>(k) * Rp + c) * M + m] = {0, 0};
                    if (proj_dh != nullptr) proj_dh[(static_cast<size_t>(k) * Rp + c) * M + m] = {0, 0};
                }
        }
    }
}

__global__ void k_init_rho(int Rp, int G, const c128 *partial, ColState cs) {
    __shared__ c128 lds[kBlock];
    const int c = blockIdx.x;
    c128 v{0, 0};
    for (int g = threadIdx.x; g < G; g += kBlock) v = v + partial[static_cast<size_t>(g) * Rp + c];
    const c128 rho = block_sum(v, lds);
    if (threadIdx.x == 0 && !cs.done[c]) {
        cs.rho[c] = rho;
        if (!cfinite(rho)) { cs.flags[c] |= FLAG_NAN; cs.done[c] = 1; }
        else if (cabs(rho) == 0.0) { cs.flags[c] |= FLAG_BREAKDOWN; cs.done[c] = 1; }
    }
}

// Extreme Ritz values of the Lanczos tridiagonal that a recorded CG solve
// (step sizes a_j, ratios b_j) builds implicitly:
//   T_00 = 1/a_0,  T_jj = 1/a_j + b_{j-1}/a_{j-1},  T_{j,j+1} = sqrt(b_j)/a_j,
// found by bisection on the Sturm count.  One thread per column.
__device__ inline int sturm_below(const double *dg, const double *of, int k, double x) {
    int cnt = 0;
    double q = dg[0] - x;
    if (q < 0) ++cnt;
    for (int j = 1; j < k; ++j) {
        const double qq = (q == 0.0) ? 1e-300 : q;
        q = (dg[j] - x) - of[j - 1] * of[j - 1] / qq;
        if (q < 0) ++cnt;
    }
    return cnt;
}

__global__ void k_ritz(int R, int Rp, ColState cs, double *lmin, double *lmax) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Rp) return;
    lmin[c] = 1e300;
    lmax[c] = -1e300;
    if (c >= R || cs.zres[c] || cs.done[c]) return;
    const int k = min(cs.inner_count[c], kHist);
    if (k < 1) return;
    double dg[kHist], of[kHist];
    const double *a = cs.cg_ha + static_cast<size_t>(c) * kHist;
    const double *b = cs.cg_hb + static_cast<size_t>(c) * kHist;
    for (int j = 0; j < k; ++j) {
        dg[j] = 1.0 / a[j] + (j > 0 ? b[j - 1] / a[j - 1] : 0.0);
        of[j] = j + 1 < k ? sqrt(b[j]) / a[j] : 0.0;
    }
    double lo = 1e300, hi = -1e300;
    for (int j = 0; j < k; ++j) {
        const double rad = (j > 0 ? fabs(of[j - 1]) : 0.0) + (j + 1 < k ? fabs(of[j]) : 0.0);
        lo = fmin(lo, dg[j] - rad);
        hi = fmax(hi, dg[j] + rad);
    }
    // smallest eigenvalue: largest x with no eigenvalue below it
    double x0 = lo, x1 = hi;
    for (int it = 0; it < 100; ++it) {
        const double m = 0.5 * (x0 + x1);
        if (sturm_below(dg, of, k, m) >= 1) x1 = m; else x0 = m;
    }
    lmin[c] = x0;
    x0 = lo; x1 = hi;
    for (int it = 0; it < 100; ++it) {
        const double m = 0.5 * (x0 + x1);
        if (sturm_below(dg, of, k, m) >= k) x1 = m; else x0 = m;
    }
    lmax[c] = x1;
}

__global__ void k_ritz_reduce(int Rp, const double *lmin, const double *lmax, double *out) {
    __shared__ double a[kBlock], b[kBlock];
    double mn = 1e300, mx = -1e300;
    for (int c = threadIdx.x; c < Rp; c += kBlock) { mn = fmin(mn, lmin[c]); mx = fmax(mx, lmax[c]); }
    a[threadIdx.x] = mn;
    b[threadIdx.x] = mx;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            a[threadIdx.x] = fmin(a[threadIdx.x], a[threadIdx.x + s]);
            b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = a[0]; out[1] = b[0]; }
}

// Residual check of the Chebyshev iteration: a column is finished when
// ||r - S y|| <= thr * ||r|| (inner_done = 1), else it needs more steps.
__global__ __launch_bounds__(kBlock) void k_cheb_check(int Rp, int G, const double *partial, double thr,
                                                       int final_check, ColState cs) {
    __shared__ double lds[kBlock];
    const int c = blockIdx.x;
    if (cs.done[c] || cs.inner_done[c]) return;
    double v = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) v += partial[static_cast<size_t>(g) * Rp + c];
    const double rr = block_sum(v, lds);
    if (threadIdx.x != 0) return;
    if (!isfinite(rr)) { cs.flags[c] |= FLAG_NAN; cs.done[c] = 1; cs.inner_done[c] = 1; return; }
    if (rr <= thr * thr * cs.rnorm2[c]) {
        cs.inner_done[c] = 1;
    } else if (final_check) {
        cs.flags[c] |= FLAG_INNER;   // inexact S^{-1} r for this column this iteration
        cs.inner_done[c] = 1;
    }
}

template <typename T>
__global__ void k_copy_vec(size_t n, const cpx<T> *a, cpx<T> *b) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_to_c64(size_t n, const c128 *a, c64 *b) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = ccast<float>(a[i]);
}

__global__ void k_status(int Rp, ColState cs, Status *st) {
    __shared__ int a[kBlock], b[kBlock], s[kBlock], f[kBlock];
    __shared__ double wr[kBlock];
    __shared__ long long it[kBlock];
    int na = 0, nb = 0, ns = 0, fl = 0;
    double w = -1.0;
    long long ni = 0;
    for (int c = threadIdx.x; c < Rp; c += kBlock) {
        const int done = cs.done[c];
        na += !done;
        nb += (!done && !cs.inner_done[c]);
        ns += (!done && cs.sw[c] != 0);
        fl |= cs.flags[c];
        if (!done) w = fmax(w, cs.wres[c]);
        ni += cs.iters[c];
    }
    a[threadIdx.x] = na; b[threadIdx.x] = nb; s[threadIdx.x] = ns; f[threadIdx.x] = fl; wr[threadIdx.x] = w;
    it[threadIdx.x] = ni;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            a[threadIdx.x] += a[threadIdx.x + k];
            b[threadIdx.x] += b[threadIdx.x + k];
            s[threadIdx.x] += s[threadIdx.x + k];
            f[threadIdx.x] |= f[threadIdx.x + k];
            wr[threadIdx.x] = fmax(wr[threadIdx.x], wr[threadIdx.x + k]);
            it[threadIdx.x] += it[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->active_cols = a[0];
        st->inner_pending = b[0];
        st->switched = s[0];
        st->flags = f[0];
        st->worst_res = wr[0];
        st->col_iters = it[0];
    }
}

// ------------------------------------------------------------------ vector kernels
// r <- r - alpha q; r32 (if given) receives r in complex64: the right-hand
// side of the first complex64 round of the mixed inner solve
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_r(int N, int Rp, int Lr, const int *done,
                                                     const c128 *alpha, const cpx<T> *q, cpx<T> *r,
                                                     cpx<T> *res, cpx<T> *d, double *partial, int copy,
                                                     c64 *r32) {
    ELEM_LOOP_BEGIN
    double acc = 0.0;
    if (!done[col]) {
        const cpx<T> a = ccast<T>(alpha[col]);
        for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
            const size_t e = static_cast<size_t>(i) * Rp + col;
            const cpx<T> v = r[e] - a * q[e];
            r[e] = v;
            if (r32) r32[e] = ccast<float>(v);
            if (copy) {
                // starting residual and direction of a CG inner solve
                res[e] = v;
                d[e] = v;
            }
            acc += static_cast<double>(v.re) * v.re + static_cast<double>(v.im) * v.im;
        }
    }
    wave_partial_store(acc, partial, g, Rp, col);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(int N, int Rp, int Lr, const int *inner_done,
                                                      const int *first, const double *cg_a,
                                                      const cpx<T> *d, const cpx<T> *w, cpx<T> *y,
                                                      cpx<T> *res, double *partial) {
    ELEM_LOOP_BEGIN
    double acc = 0.0;
    if (!inner_done[col]) {
        const T a = static_cast<T>(cg_a[col]);
        const bool f = first[col] != 0;
        for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
            const size_t e = static_cast<size_t>(i) * Rp + col;
            const cpx<T> dv = d[e];
            const cpx<T> yv = f ? a * dv : y[e] + a * dv;
            y[e] = yv;
            const cpx<T> rv = res[e] - a * w[e];
            res[e] = rv;
            acc += static_cast<double>(rv.re) * rv.re + static_cast<double>(rv.im) * rv.im;
        }
    }
    wave_partial_store(acc, partial, g, Rp, col);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_dir(int N, int Rp, int Lr, const int *inner_done,
                                                   const double *cg_b, const cpx<T> *res, cpx<T> *d) {
    ELEM_LOOP_BEGIN
    if (inner_done[col]) return;
    const T b = static_cast<T>(cg_b[col]);
    for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
        const size_t e = static_cast<size_t>(i) * Rp + col;
        d[e] = res[e] + b * d[e];
    }
}

// partial r'^T r (unconjugated)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rho_dot(int N, int Rp, int Lr, const int *done, const int *zres,
                                                    const cpx<T> *rp, const cpx<T> *r, c128 *partial) {
    ELEM_LOOP_BEGIN
    c128 acc{0, 0};
    if (!done[col] && !zres[col]) {
        for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
            const size_t e = static_cast<size_t>(i) * Rp + col;
            acc = acc + ccast<double>(rp[e]) * ccast<double>(r[e]);
        }
    }
    wave_partial_store(acc, partial, g, Rp, col);
}

// p <- r' + beta p (eq. CGp:p); at a seed switch p <- r'/c + beta p^{s'} with
// r, r' rescaled by 1/c; at a collinear restart (or init) p <- r'.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_p_update(int N, int Rp, int Lr, int init, ColState cs,
                                                     cpx<T> *rp, cpx<T> *r, cpx<T> *p, const cpx<T> *P,
                                                     size_t ldk, cpx<T> *ringT) {
    // ringT (optional): the block's Lr x 64 tile of the (rescaled) r' is also
    // written column-major through LDS, for the fused shift update
    extern __shared__ unsigned char tile_raw[];
    cpx<T> *tile = reinterpret_cast<cpx<T> *>(tile_raw);
    ELEM_LOOP_BEGIN
    const bool active = !cs.done[col];
    const int sw = init ? 2 : cs.sw[col];
    const cpx<T> beta = ccast<T>(cs.beta_prev[col]);
    const int tl = Lr + 1;
    if (active && sw == 1) {
        const c128 cc = cs.swc[col];
        const c128 inv = cdiv(c128{1.0, 0.0}, cc);
        const cpx<T> ci = ccast<T>(inv);
        const cpx<T> *Ps = P + static_cast<size_t>(cs.seed[col]) * ldk + static_cast<size_t>(col) * N;
        for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
            const size_t e = static_cast<size_t>(i) * Rp + col;
            const cpx<T> v = ci * rp[e];
            rp[e] = v;
            r[e] = ci * r[e];
            p[e] = v + beta * Ps[i];
            if (ringT) tile[lane * tl + (i - i0)] = v;
        }
    } else if (active && sw == 2) {
        for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
            const size_t e = static_cast<size_t>(i) * Rp + col;
            const cpx<T> v = rp[e];
            p[e] = v;
            if (ringT) tile[lane * tl + (i - i0)] = v;
        }
    } else if (active) {
        for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
            const size_t e = static_cast<size_t>(i) * Rp + col;
            const cpx<T> v = rp[e];
            p[e] = v + beta * p[e];
            if (ringT) tile[lane * tl + (i - i0)] = v;
        }
    }
    if (ringT == nullptr) return;
    __syncthreads();
    const int rows = i1 - i0;
    const int c0 = cx * 64;
    for (int t = threadIdx.x; t < 64 * rows; t += kBlock) {
        const int c = t / rows, row = t % rows;
        ringT[static_cast<size_t>(c0 + c) * N + i0 + row] = tile[c * tl + row];
    }
}

// Column-major copy of one r' ring slot: dst[c][i] = src[i][c].  The fused
// shift update walks one column's rows, which this layout makes contiguous.
// Tile of 32 rows x 64 columns through LDS (row stride padded by one).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ring_transpose(int N, int Rp, const cpx<T> *__restrict__ src,
                                                           cpx<T> *__restrict__ dst) {
    __shared__ cpx<T> tile[64][33];
    const int c0 = blockIdx.x * 64;
    const int t = threadIdx.x;
    // 32-row tiles, strided over the grid's second dimension (uniform trip
    // count per block, so the barriers are reached by every thread)
    for (int r0 = blockIdx.y * 32; r0 < N; r0 += gridDim.y * 32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = t & 63, r = (t >> 6) + 4 * j;
            if (r0 + r < N) tile[c][r] = src[static_cast<size_t>(r0 + r) * Rp + c0 + c];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = t & 31, c = (t >> 5) + 8 * j;
            if (r0 + r < N) dst[static_cast<size_t>(c0 + c) * N + r0 + r] = tile[c][r];
        }
        __syncthreads();
    }
}

__global__ void k_mark_applied(int Rp, int n1, ColState cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < Rp && cs.sw[c] == 1) cs.applied[c] = n1;
}

// ------------------------------------------------------------------ fused shift update
__device__ inline double readlane_f64(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffull), l));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), l));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}
__device__ inline c128 readlane_c128(c128 v, int l) { return {readlane_f64(v.re, l), readlane_f64(v.im, l)}; }

// The update coefficients of steps [tb, tb + M) of shift k, column col, one
// per lane: lane w*M + j holds coefficient w (0: a, 1: b, 2: c) of step
// tb + j.  One vector load per shift (contiguous [Rp][K][m] layout).
template <int M>
__device__ inline c128 load_coefs(const ShiftState &ss, int k, int col, int tb, int cnt, int m) {
    const int lane = threadIdx.x & 63;
    const int w = lane / M, j = lane % M;
    if (w >= 3 || j >= cnt) return {0, 0};
    const c128 *arr = w == 0 ? ss.ra : w == 1 ? ss.rb : ss.rc;
    return arr[coef_at(ss, k, col, (tb + j) % m)];
}

// Walks the shifts of one column that still take steps in a pass, 64 at a
// time: lane l holds the step count of shift q*64 + l, and a ballot gives
// the active ones, so frozen shifts cost nothing.
struct ActiveShifts {
    int K, Rp, col, tb, n1, q = -1, st = 0;
    unsigned long long mask = 0;
    const int *last;
    // next active shift (k, its step count) or k = -1
    __device__ inline void next(int &k, int &kc) {
        while (mask == 0) {
            if ((q + 1) * 64 >= K) { k = -1; kc = 0; return; }
            ++q;
            const int kk = q * 64 + static_cast<int>(threadIdx.x & 63);
            st = 0;
            if (kk < K) {
                const int l = last[static_cast<size_t>(kk) * Rp + col];
                st = (l >= n1 ? n1 : l + 1) - tb;
            }
            mask = __ballot(st > 0);
        }
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        k = q * 64 + b;
        kc = __builtin_amdgcn_readlane(st, b);
    }
};

// Applies the pending steps t in [max(n0, applied[c]), n1) of the shifted
// recurrences to x^k, p^k of column c:  p <- a_t r'_t + b_t p;  x <- x + c_t p,
// skipping shifts that froze before the pass and steps after a shift froze.
// r'_t stays in registers across all shifts of the column (read from the
// column-major copy of the ring); x^k, p^k are read and written once per
// pass.  The next active shift's rows and coefficients are in flight while
// the current one is updated.
template <typename T, int M, int E>
__global__ __launch_bounds__(kBlock) void k_flush(int N, int Rp, int K, int m, int n0, int n1, int only_sw,
                                                  ColState cs, ShiftState ss,
                                                  const cpx<T> *__restrict__ ringT, size_t ring_ld,
                                                  cpx<T> *__restrict__ X, size_t ldx, cpx<T> *__restrict__ P,
                                                  size_t ldp, int R) {
    const int rc = blockIdx.x;
    const int col = blockIdx.y;
    if (col >= R) return;
    if (only_sw && cs.sw[col] != 1) return;
    if (cs.iters[col] == 0) return;   // b = 0: the column never took a step, x^k = 0
    const int tb = max(n0, cs.applied[col]);
    const int cnt = n1 - tb;
    if (cnt <= 0) return;
    // a pass from step 0 is the column's first: x^k = p^k = 0 before it, so
    // they are not read (nor zeroed beforehand)
    const bool fresh = tb == 0;
    ActiveShifts act{K, Rp, col, tb, n1};
    act.last = ss.last;
    int k, kc;
    act.next(k, kc);
    if (k < 0) return;
    const int ibase = rc * (kBlock * E) + threadIdx.x;
    const size_t base = static_cast<size_t>(col) * N;
    auto load_rows = [&](int kk, cpx<T> (&pv)[E], cpx<T> (&xv)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = ibase + e * kBlock;
            pv[e] = (i < N && !fresh) ? P[static_cast<size_t>(kk) * ldp + base + i] : cpx<T>{0, 0};
            xv[e] = (i < N && !fresh) ? X[static_cast<size_t>(kk) * ldx + base + i] : cpx<T>{0, 0};
        }
    };
    cpx<T> pv[E], xv[E];
    load_rows(k, pv, xv);
    c128 cf = load_coefs<M>(ss, k, col, tb, cnt, m);
    cpx<T> rr[M][E];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const int slot = (tb + j) % m;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = ibase + e * kBlock;
            rr[j][e] = (j < cnt && i < N) ? ringT[slot * ring_ld + static_cast<size_t>(col) * N + i]
                                          : cpx<T>{0, 0};
        }
    }
    while (k >= 0) {
        int kn, kcn;
        act.next(kn, kcn);
        cpx<T> pn[E], xn[E];
        c128 cfn{0, 0};
        if (kn >= 0) {
            load_rows(kn, pn, xn);
            cfn = load_coefs<M>(ss, kn, col, tb, cnt, m);
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < kc) {
                const cpx<T> a = ccast<T>(readlane_c128(cf, j));
                const cpx<T> b = ccast<T>(readlane_c128(cf, M + j));
                const cpx<T> cc = ccast<T>(readlane_c128(cf, 2 * M + j));
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    pv[e] = a * rr[j][e] + b * pv[e];
                    xv[e] = xv[e] + cc * pv[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = ibase + e * kBlock;
            if (i < N) {
                P[static_cast<size_t>(k) * ldp + base + i] = pv[e];
                X[static_cast<size_t>(k) * ldx + base + i] = xv[e];
            }
        }
        if (kn < 0) break;
#pragma unroll
        for (int e = 0; e < E; ++e) { pv[e] = pn[e]; xv[e] = xn[e]; }
        cf = cfn;
        k = kn;
        kc = kcn;
    }
}

// ------------------------------------------------------------------ projected carry
// g_{k,m} += c^k h_{k,m},  h_{k,m} <- a^k (c_m^T r') + b^k h_{k,m}  for the
// projections c_m = e_{idx} (unit) and optionally c = S e_a, a = rhs[c] (srow).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_update(int K, int Rp, int Mu, int srow, int slot, int B,
                                                        const int32_t *rowptr, const int32_t *colidx,
                                                        const double *Sval, const int64_t *rhs,
                                                        const int32_t *pidx, ColState cs, ShiftState ss,
                                                        const cpx<T> *rp, c128 *h, c128 *gacc) {
    extern __shared__ c128 cr[];
    const int c = blockIdx.x;
    if (cs.done[c]) return;
    const int M = Mu + srow;
    for (int m = threadIdx.x; m < Mu; m += kBlock)
        cr[m] = ccast<double>(rp[static_cast<size_t>(pidx[static_cast<size_t>(c) * Mu + m]) * Rp + c]);
    if (srow) {
        __shared__ c128 lds[kBlock];
        const int64_t a = rhs[c];
        const int I = static_cast<int>(a / B), ar = static_cast<int>(a % B);
        const int b0 = rowptr[I], b1 = rowptr[I + 1];
        c128 acc{0, 0};
        for (int t = threadIdx.x; t < (b1 - b0) * B; t += kBlock) {
            const int b = b0 + t / B, cc = t % B;
            const double s = Sval[(static_cast<size_t>(b) * B + ar) * B + cc];
            acc = acc + s * ccast<double>(rp[static_cast<size_t>(colidx[b] * B + cc) * Rp + c]);
        }
        const c128 tot = block_sum(acc, lds);
        if (threadIdx.x == 0) cr[Mu] = tot;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < K * M; t += kBlock) {
        const int k = t / M, m = t % M;
        const size_t idx = static_cast<size_t>(k) * Rp + c;
        if (ss.last[idx] != kFrozenNever) continue;
        const size_t s = coef_at(ss, k, c, slot);
        const size_t o = idx * M + m;
        const c128 hv = ss.ra[s] * cr[m] + ss.rb[s] * h[o];
        h[o] = hv;
        gacc[o] = gacc[o] + ss.rc[s] * hv;
    }
}

// Projected carry with the z-derivative, accumulating the quadrature-weighted
// sums the band-energy gradient needs (wE_k = w_k Re z_k):
//   AG_m += wE_k  dG_{k,m},   AD_m += wE_k  d(dG)_{k,m},   AZ_m += wE_k z_k d(dG)_{k,m}
// where dG_{k,m} is this step's increment of c_m^T x^k and d(dG) that of its
// z-derivative.  One thread per projection m loops over the shifts, so each
// accumulator has a single owner (no reduction, deterministic).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_update_vjp(
    int K, int Rp, int Mu, int srow, int slot, int B, const int32_t *rowptr, const int32_t *colidx,
    const double *Sval, const int64_t *rhs, const int32_t *pidx, ColState cs, ShiftState ss, const cpx<T> *rp,
    c128 *h, c128 *dh, const double *wE, c128 *acc) {
    extern __shared__ c128 cr[];
    const int c = blockIdx.x;
    if (cs.done[c]) return;
    const int M = Mu + srow;
    for (int m = threadIdx.x; m < Mu; m += kBlock)
        cr[m] = ccast<double>(rp[static_cast<size_t>(pidx[static_cast<size_t>(c) * Mu + m]) * Rp + c]);
    if (srow) {
        __shared__ c128 lds[kBlock];
        const int64_t a = rhs[c];
        const int I = static_cast<int>(a / B), ar = static_cast<int>(a % B);
        const int b0 = rowptr[I], b1 = rowptr[I + 1];
        c128 sacc{0, 0};
        for (int t = threadIdx.x; t < (b1 - b0) * B; t += kBlock) {
            const int b = b0 + t / B, cc = t % B;
            sacc = sacc + Sval[(static_cast<size_t>(b) * B + ar) * B + cc] *
                              ccast<double>(rp[static_cast<size_t>(colidx[b] * B + cc) * Rp + c]);
        }
        const c128 tot = block_sum(sacc, lds);
        if (threadIdx.x == 0) cr[Mu] = tot;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += kBlock) {
        const c128 crm = cr[m];
        c128 ag{0, 0}, ad{0, 0}, az{0, 0};
        for (int k = 0; k < K; ++k) {
            const size_t idx = static_cast<size_t>(k) * Rp + c;
            if (ss.last[idx] != kFrozenNever) continue;
            const size_t sidx = coef_at(ss, k, c, slot);
            const size_t o = idx * M + m;
            const c128 hold = h[o], dhold = dh[o];
            const c128 hv = ss.ra[sidx] * crm + ss.rb[sidx] * hold;
            const c128 dhv = ss.rda[sidx] * crm + ss.rdb[sidx] * hold + ss.rb[sidx] * dhold;
            h[o] = hv;
            dh[o] = dhv;
            const c128 dg = ss.rc[sidx] * hv;
            const c128 ddg = ss.rdc[sidx] * hv + ss.rc[sidx] * dhv;
            const double we = wE[k];
            ag = ag + we * dg;
            ad = ad + we * ddg;
            az = az + we * (ss.z[k] * ddg);
        }
        c128 *A = acc + (static_cast<size_t>(c) * M + m) * 3;
        A[0] = A[0] + ag;
        A[1] = A[1] + ad;
        A[2] = A[2] + az;
    }
}

// ------------------------------------------------------------------ outputs
// (S x^k)_a for unit rhs a = rhs[c] from the full-carry iterates.
template <typename T>
__global__ void k_sx_diag(int K, int R, int N, int B, const int32_t *rowptr, const int32_t *colidx,
                          const double *Sval, const int64_t *rhs, const cpx<T> *X, size_t ldk,
                          c128 *out, int ldo, int r0) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(K) * R) return;
    const int k = static_cast<int>(t / R), c = static_cast<int>(t % R);
    const int64_t a = rhs[c];
    const int I = static_cast<int>(a / B), ar = static_cast<int>(a % B);
    const cpx<T> *x = X + static_cast<size_t>(k) * ldk + static_cast<size_t>(c) * N;
    c128 acc{0, 0};
    for (int b = rowptr[I]; b < rowptr[I + 1]; ++b)
        for (int cc = 0; cc < B; ++cc)
            acc = acc + Sval[(static_cast<size_t>(b) * B + ar) * B + cc] * ccast<double>(x[colidx[b] * B + cc]);
    out[static_cast<size_t>(k) * ldo + r0 + c] = acc;
}

template <typename T>
__global__ void k_gather_proj(int K, int R, int N, int np, const int32_t *pidx, const cpx<T> *X, size_t ldk,
                              c128 *out, int nrhs_total, int r0) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(K) * R * np) return;
    const int m = static_cast<int>(t % np);
    const int c = static_cast<int>((t / np) % R);
    const int k = static_cast<int>(t / (static_cast<int64_t>(np) * R));
    const int i = pidx[static_cast<size_t>(c) * np + m];
    out[(static_cast<size_t>(k) * nrhs_total + r0 + c) * np + m] =
        ccast<double>(X[static_cast<size_t>(k) * ldk + static_cast<size_t>(c) * N + i]);
}

// copy / widen the tile's x^k into the caller's [K][nrhs][N] complex128 layout
template <typename T>
__global__ void k_store_cols(int K, int R, int N, const cpx<T> *X, size_t ldk, c128 *out, int nrhs_total,
                             int r0) {
    const int64_t per = static_cast<int64_t>(R) * N;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= per * K) return;
    const int64_t k = t / per, o = t % per;
    out[(k * nrhs_total + r0) * N + o] = ccast<double>(X[k * ldk + o]);
}

__global__ void k_store_proj(int K, int R, int Rp, int M, const c128 *g, c128 *out, int nrhs_total, int r0) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(K) * R * M) return;
    const int m = static_cast<int>(t % M);
    const int c = static_cast<int>((t / M) % R);
    const int k = static_cast<int>(t / (static_cast<int64_t>(M) * R));
    out[(static_cast<size_t>(k) * nrhs_total + r0 + c) * M + m] = g[(static_cast<size_t>(k) * Rp + c) * M + m];
}

// FP64 true residual ||b - (z_k S - H) x_k||^2 (partial per (k, c) by rows)
template <typename T>
__global__ void k_true_residual(int K, int R, int N, int B, const int32_t *rowptr, const int32_t *colidx,
                                const double *Sval, const double *Hval, const c128 *z, const int64_t *rhs,
                                const c128 *Bd, const cpx<T> *X, size_t ldk, double *out) {
    // one block per (k, c); threads stride rows
    __shared__ double lds[kBlock];
    const int k = blockIdx.y, c = blockIdx.x;
    const cpx<T> *x = X + static_cast<size_t>(k) * ldk + static_cast<size_t>(c) * N;
    const c128 zk = z[k];
    double acc = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) {
        const int I = i / B, ar = i % B;
        c128 s{0, 0}, h{0, 0};
        for (int b = rowptr[I]; b < rowptr[I + 1]; ++b)
            for (int cc = 0; cc < B; ++cc) {
                const c128 xv = ccast<double>(x[colidx[b] * B + cc]);
                s = s + Sval[(static_cast<size_t>(b) * B + ar) * B + cc] * xv;
                h = h + Hval[(static_cast<size_t>(b) * B + ar) * B + cc] * xv;
            }
        c128 bv{0, 0};
        if (rhs != nullptr) bv = (i == rhs[c]) ? c128{1, 0} : c128{0, 0};
        else bv = Bd[static_cast<size_t>(c) * N + i];
        const c128 rv = bv - (zk * s - h);
        acc += cabs2(rv);
        bb += cabs2(bv);
    }
    const double ta = block_sum(acc, lds);
    const double tb = block_sum(bb, lds);
    // b = 0: x = 0 is exact (relative residual 0)
    if (threadIdx.x == 0) out[static_cast<size_t>(k) * R + c] = tb > 0.0 ? sqrt(ta) / sqrt(tb) : sqrt(ta);
}

// ------------------------------------------------------------------ driver
namespace {

// ------------------------------------------------------------------ generalised Lanczos
// Sec. 3.2, eqs. 1.13 and 1.18: the S-orthonormal three-term recursion of
// M = S^{-1} H started at S^{-1} e_j, and G_jj(z) from its continued
// fraction.  The Lanczos vectors are real: process p = 2c + q lives in part
// q (0 real, 1 imaginary) of column c, so the products and the inner
// S-solve act on two processes at once and only the dots are split.

// sums over the 4 waves of a block, two values per lane -> two partial planes
__device__ inline void wave_partial_store2(double v0, double v1, double *part, int G, int g, int Rp, int col) {
    __shared__ double red[2][kWavesPerBlock][64];
    const int lane = threadIdx.x & 63;
    red[0][threadIdx.x >> 6][lane] = v0;
    red[1][threadIdx.x >> 6][lane] = v1;
    __syncthreads();
    if (threadIdx.x < 64) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) { s0 += red[0][k][lane]; s1 += red[1][k][lane]; }
        part[static_cast<size_t>(g) * Rp + col] = s0;
        part[(static_cast<size_t>(G) + g) * Rp + col] = s1;
    }
}

// r = e_j in each process's part (res = d = r for a CG start), partial |r|^2
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_unit(int N, int Rp, int Lr, int P, const int64_t *rhs, cpx<T> *r,
                                                    cpx<T> *res, cpx<T> *d, double *partial) {
    ELEM_LOOP_BEGIN
    const int64_t jr = 2 * col < P ? rhs[2 * col] : -1;
    const int64_t ji = 2 * col + 1 < P ? rhs[2 * col + 1] : -1;
    double acc = 0.0;
    for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
        const cpx<T> v{i == jr ? T(1) : T(0), i == ji ? T(1) : T(0)};
        const size_t e = static_cast<size_t>(i) * Rp + col;
        r[e] = v;
        res[e] = v;
        d[e] = v;
        acc += static_cast<double>(v.re) * v.re + static_cast<double>(v.im) * v.im;
    }
    wave_partial_store(acc, partial, g, Rp, col);
}

// v_j = (S^{-1} e_j)_j = ||S^{-1} e_j||_S^2 of every process, 1/sqrt(v_j), and
// the process state (a process without a right-hand side is finished)
template <typename T>
__global__ void k_lz_vj(int P, int Rp, const int64_t *rhs, const cpx<T> *v, double *vj, double *inv, int *steps,
                        int *done) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= 2 * Rp) return;
    double val = 0.0;
    if (p < P) {
        const cpx<T> x = v[static_cast<size_t>(rhs[p]) * Rp + (p >> 1)];
        val = (p & 1) ? x.im : x.re;
    }
    const bool ok = p < P && val > 0.0 && isfinite(val);
    vj[p] = ok ? val : 0.0;
    inv[p] = ok ? 1.0 / sqrt(val) : 0.0;
    steps[p] = 0;
    done[p] = ok ? 0 : 1;
}

// u^0 = v / sqrt(v_j), u^{-1} = 0 and S u^{-1} = 0 (S u^n is formed by the
// product of each step)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_start(int N, int Rp, int Lr, const double *inv, const cpx<T> *v,
                                                     cpx<T> *u, cpx<T> *up, cpx<T> *sp) {
    ELEM_LOOP_BEGIN
    const T ir = static_cast<T>(inv[2 * col]), ii = static_cast<T>(inv[2 * col + 1]);
    for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
        const size_t e = static_cast<size_t>(i) * Rp + col;
        const cpx<T> x = v[e];
        u[e] = {x.re * ir, x.im * ii};
        up[e] = {0, 0};
        sp[e] = {0, 0};
    }
}

// a_n = u^T H u of both processes of a column from the product's partials
__global__ __launch_bounds__(kBlock) void k_lz_reduce_a(int Rp, int Gs, const double *part, int n, int mmax,
                                                        double *a, int *steps, const int *done) {
    __shared__ double lds[kBlock];
    const int c = blockIdx.x;
    double s0 = 0.0, s1 = 0.0;
    for (int g = threadIdx.x; g < Gs; g += kBlock) {
        s0 += part[static_cast<size_t>(g) * Rp + c];
        s1 += part[(static_cast<size_t>(Gs) + g) * Rp + c];
    }
    s0 = block_sum(s0, lds);
    s1 = block_sum(s1, lds);
    if (threadIdx.x != 0) return;
    for (int q = 0; q < 2; ++q) {
        const int p = 2 * c + q;
        if (done[p]) continue;
        a[static_cast<size_t>(p) * mmax + n] = q ? s1 : s0;
        steps[p] = n + 1;
    }
}

// w' = w - a_n u - b_n u^{n-1} (over w) and the partial w'^T S w' of both
// parts, with S w' = h - a_n S u - b_n S u^{n-1} (h = H u = S w up to the
// inner solve's tolerance; S u and S u^{n-1} are the products' fresh values)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_update(int N, int Rp, int Lr, int G, int n, int mmax, const double *a,
                                                      const double *b, cpx<T> *w, const cpx<T> *u,
                                                      const cpx<T> *up, const cpx<T> *h, const cpx<T> *s,
                                                      const cpx<T> *sp, double *part) {
    ELEM_LOOP_BEGIN
    const size_t pr = static_cast<size_t>(2 * col) * mmax, pi = pr + mmax;
    const T ar = static_cast<T>(a[pr + n]), ai = static_cast<T>(a[pi + n]);
    const T br = n > 0 ? static_cast<T>(b[pr + n]) : T(0), bi = n > 0 ? static_cast<T>(b[pi + n]) : T(0);
    double acc0 = 0.0, acc1 = 0.0;
    for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
        const size_t e = static_cast<size_t>(i) * Rp + col;
        const cpx<T> uv = u[e], upv = up[e], sv = s[e], spv = sp[e], wv_ = w[e], hv = h[e];
        const cpx<T> wn{wv_.re - ar * uv.re - br * upv.re, wv_.im - ai * uv.im - bi * upv.im};
        const cpx<T> sn{hv.re - ar * sv.re - br * spv.re, hv.im - ai * sv.im - bi * spv.im};
        w[e] = wn;
        acc0 += static_cast<double>(wn.re) * sn.re;
        acc1 += static_cast<double>(wn.im) * sn.im;
    }
    wave_partial_store2(acc0, acc1, part, G, g, Rp, col);
}

// b_{n+1} = ||w'||_S and 1/b_{n+1} per process; a finished process, or one
// whose Krylov space is exhausted (b_{n+1} ~ 0), gets 1/b = 0 (its vectors
// become zero and stay zero)
__global__ __launch_bounds__(kBlock) void k_lz_reduce_b(int Rp, int G, const double *part, int n, int mmax,
                                                        const double *a, double *b, double *inv, int *done) {
    __shared__ double lds[kBlock];
    const int c = blockIdx.x;
    double s0 = 0.0, s1 = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) {
        s0 += part[static_cast<size_t>(g) * Rp + c];
        s1 += part[(static_cast<size_t>(G) + g) * Rp + c];
    }
    s0 = block_sum(s0, lds);
    s1 = block_sum(s1, lds);
    if (threadIdx.x != 0) return;
    for (int q = 0; q < 2; ++q) {
        const int p = 2 * c + q;
        if (done[p]) { inv[p] = 0.0; continue; }
        const double bn = sqrt(fmax(q ? s1 : s0, 0.0));
        const double an = a[static_cast<size_t>(p) * mmax + n];
        if (!(bn > 1e-14 * fmax(1.0, fabs(an))) || !isfinite(bn)) {
            done[p] = 1;
            inv[p] = 0.0;
            continue;
        }
        if (n + 1 < mmax) b[static_cast<size_t>(p) * mmax + n + 1] = bn;
        inv[p] = 1.0 / bn;
    }
}

// u^{n+1} = w' / b_{n+1}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_scale(int N, int Rp, int Lr, const double *inv, const cpx<T> *w,
                                                     cpx<T> *un) {
    ELEM_LOOP_BEGIN
    const T ir = static_cast<T>(inv[2 * col]), ii = static_cast<T>(inv[2 * col + 1]);
    for (int i = i0 + wv; i < i1; i += kWavesPerBlock) {
        const size_t e = static_cast<size_t>(i) * Rp + col;
        const cpx<T> x = w[e];
        un[e] = {x.re * ir, x.im * ii};
    }
}

// G_jj(z_k) = v_j / (z_k - a_0 - b_1^2 / (z_k - a_1 - ...)) at each process's
// current depth, evaluated from the bottom.  Check mode: compare with the
// previous check (finished when the change over all shifts is at most tol
// times the largest |G|); final mode: write G.
__global__ __launch_bounds__(kBlock) void k_lz_cf(int K, int mmax, const c128 *z, const double *a, const double *b,
                                                  const double *vj, const int *steps, c128 *gprev, double tol,
                                                  int *done, int final_, c128 *out, int ldo, int p0) {
    __shared__ double l1[kBlock], l2[kBlock];
    const int p = blockIdx.x;
    const int d = steps[p];
    const double *ap = a + static_cast<size_t>(p) * mmax, *bp = b + static_cast<size_t>(p) * mmax;
    double dmax = 0.0, gmax = 0.0;
    for (int k = threadIdx.x; k < K; k += kBlock) {
        c128 g{0.0, 0.0};
        if (d > 0 && vj[p] > 0.0) {
            const c128 zk = z[k];
            c128 t{zk.re - ap[d - 1], zk.im};
            for (int i = d - 2; i >= 0; --i) {
                const c128 q = cdiv(c128{bp[i + 1] * bp[i + 1], 0.0}, t);
                t = c128{zk.re - ap[i] - q.re, zk.im - q.im};
            }
            g = cdiv(c128{vj[p], 0.0}, t);
        }
        if (final_) {
            out[static_cast<size_t>(k) * ldo + p0 + p] = g;
        } else {
            const size_t o = static_cast<size_t>(p) * K + k;
            dmax = fmax(dmax, cabs(g - gprev[o]));
            gmax = fmax(gmax, cabs(g));
            gprev[o] = g;
        }
    }
    if (final_) return;
    l1[threadIdx.x] = dmax;
    l2[threadIdx.x] = gmax;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            l1[threadIdx.x] = fmax(l1[threadIdx.x], l1[threadIdx.x + s]);
            l2[threadIdx.x] = fmax(l2[threadIdx.x], l2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && !done[p] && l1[0] <= tol * l2[0]) done[p] = 1;
}

__global__ void k_lz_fill(size_t n, c128 v, c128 *x) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

// a column is finished when both of its processes are
__global__ void k_lz_cols(int Rp, const int *done, int *cdone) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < Rp) cdone[c] = (done[2 * c] && done[2 * c + 1]) ? 1 : 0;
}

int pick_groups(int64_t rows, int colchunks, int target_blocks) {
    int g = std::max(1, target_blocks / std::max(1, colchunks));
    g = static_cast<int>(std::min<int64_t>(g, (rows + 3) / 4));
    g = std::max(g, 1);
    g = (g + 7) / 8 * 8;
    return g;
}

template <typename T> struct Tile {
    TileDims td{};
    DevBuf<cpx<T>> p, q, r, res, d, w, ring, ringT;
    DevBuf<cpx<T>> Xown, P;
    cpx<T> *X = nullptr;
    size_t ldk = 0;
    // column state
    DevBuf<c128> c_rho, c_alpha, c_alpha_prev, c_beta_prev, c_swc, c_swcm;
    DevBuf<double> c_bnorm, c_rnorm2, c_rr, c_rr_stop, c_cg_a, c_cg_b, c_wres;
    DevBuf<int> c_seed, c_done, c_inner_done, c_cg_first, c_sw, c_applied, c_flags, c_zres, c_inner_count,
        c_iters;
    DevBuf<long long> c_shift_iters, c_inner_total, act_hist, col_hist;
    DevBuf<double> cg_ha, cg_hb;
    // shift state
    DevBuf<c128> s_pi, s_pi_prev, s_pi_next, s_omega, s_ra, s_rb, s_rc;
    DevBuf<c128> s_dpi, s_dpi_prev, s_dpi_next, s_domega, s_rda, s_rdb, s_rdc, dh;
    DevBuf<double> s_res;
    DevBuf<int> s_last;
    // partials
    DevBuf<c128> part_c;
    DevBuf<double> part_d;
    // projected carry
    DevBuf<c128> h, gacc;
    DevBuf<int32_t> pidx;
    int Mu = 0, srow = 0;

    ColState cols() {
        ColState c{};
        c.rho = c_rho.get(); c.alpha = c_alpha.get(); c.alpha_prev = c_alpha_prev.get();
        c.beta_prev = c_beta_prev.get(); c.swc = c_swc.get(); c.swcm = c_swcm.get();
        c.bnorm = c_bnorm.get(); c.rnorm2 = c_rnorm2.get(); c.rr = c_rr.get(); c.rr_stop = c_rr_stop.get();
        c.cg_a = c_cg_a.get(); c.cg_b = c_cg_b.get(); c.seed = c_seed.get(); c.done = c_done.get();
        c.inner_done = c_inner_done.get(); c.cg_first = c_cg_first.get(); c.sw = c_sw.get();
        c.applied = c_applied.get(); c.flags = c_flags.get(); c.zres = c_zres.get();
        c.inner_count = c_inner_count.get(); c.shift_iters = c_shift_iters.get(); c.iters = c_iters.get();
        c.inner_total = c_inner_total.get(); c.act_hist = act_hist.get(); c.col_hist = col_hist.get();
        c.cg_ha = cg_ha.get(); c.cg_hb = cg_hb.get(); c.wres = c_wres.get();
        return c;
    }
    ShiftState shifts(const c128 *z) {
        ShiftState s{};
        s.z = z; s.pi = s_pi.get(); s.pi_prev = s_pi_prev.get(); s.pi_next = s_pi_next.get();
        s.omega = s_omega.get(); s.res = s_res.get(); s.last = s_last.get();
        s.ra = s_ra.get(); s.rb = s_rb.get(); s.rc = s_rc.get();
        s.cK = td.K; s.cm = td.m;
        s.dpi = s_dpi.get(); s.dpi_prev = s_dpi_prev.get(); s.dpi_next = s_dpi_next.get();
        s.domega = s_domega.get(); s.rda = s_rda.get(); s.rdb = s_rdb.get(); s.rdc = s_rdc.get();
        return s;
    }
};

// Status record in pinned host memory; k_status writes it through its
// device mapping (no copy after the reduction).
struct HostStatus {
    Status *h = nullptr;
    Status *hd = nullptr;   // device address of h
    HostStatus() {
        GSC_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(Status), hipHostMallocDefault));
        GSC_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&hd), h, 0));
    }
    ~HostStatus() {
        if (h) (void)hipHostFree(h);
    }
};

template <typename T> class TileSolver {
  public:
    TileSolver(Ctx &ctx, const SolveRequest &req, const c128 *dz, const int64_t *drhs, const c128 *dB,
               int r0, int R, int Rp, int m, bool full)
        : ctx_(ctx), req_(req), pr_(*req.pair), dz_(dz), drhs_(drhs), dB_(dB), r0_(r0), full_(full) {
        auto &td = t_.td;
        td.N = static_cast<int>(pr_.n);
        td.nb = static_cast<int>(pr_.nb);
        td.B = pr_.B;
        td.K = req.K;
        td.R = R;
        td.Rp = Rp;
        td.m = m;
        td.G = pick_groups(td.N, Rp / 64, 2048);
        td.Lr = div_up(td.N, td.G);
        {
            // columns per Chebyshev launch: all steps of the inner solve run
            // on one column block at a time, sized so that the three vectors
            // the step streams (y_k, y_{k-1}, r) stay in the 256 MB infinity
            // cache between steps and the gather's re-reads hit it; blocks
            // of at least two 64-column chunks, row layout only
            const bool autob = req.opts.cheb_block <= 0;
            int cb = autob ? static_cast<int>(kChebBlockBytes / (3.0 * td.N * sizeof(cpx<T>))) / 64 * 64
                           : req.opts.cheb_block;
            // when even two chunks overflow the cache, one 64-column chunk
            // per launch: all XCDs then gather from the same x, and the
            // streamed vectors are loaded and stored nontemporal so that x
            // stays resident (measured on N = 131072: 1.94 -> 2.50 TB/s)
            const bool huge = autob && cb < 128;
            if (huge) cb = 64;
            td.cb = (cb >= 64 && cb < Rp) ? cb : Rp;
            set_spmm_geometry(td, pr_);
            if (req.opts.row_groups > 0) {
                // caller's row groups, at most one block row per wave
                const int cap = (td.nb + 3) / 4;
                td.Gs = (std::min(req.opts.row_groups, cap) + 7) / 8 * 8;
            }
            td.nt = req.opts.stream_hint == 2 || (req.opts.stream_hint == 0 && huge);
        }
        st_ = ctx_.stream;
        mixed_ = std::is_same<T, double>::value && req.opts.precision == GSC_MIXED;
        if (ctx_.prof.on) {
            const int mi = std::max(1, req.opts.max_iter);
            t_.act_hist.alloc(mi);
            t_.col_hist.alloc(mi);
            GSC_HIP(hipMemsetAsync(t_.act_hist.get(), 0, mi * sizeof(long long), st_));
            GSC_HIP(hipMemsetAsync(t_.col_hist.get(), 0, mi * sizeof(long long), st_));
        }
    }

    void allocate() {
        auto &td = t_.td;
        const size_t NR = static_cast<size_t>(td.N) * td.Rp;
        t_.p.alloc(NR); t_.q.alloc(NR); t_.r.alloc(NR); t_.res.alloc(NR); t_.d.alloc(NR); t_.w.alloc(NR);
        t_.ring.alloc(NR * td.m);
        if (full_) t_.ringT.alloc(NR * td.m);
        if (mixed_) { mx_f_.alloc(NR); mx_ya_.alloc(NR); mx_yb_.alloc(NR); }
        const size_t Rp = td.Rp;
        t_.c_rho.alloc(Rp); t_.c_alpha.alloc(Rp); t_.c_alpha_prev.alloc(Rp); t_.c_beta_prev.alloc(Rp);
        t_.c_swc.alloc(Rp); t_.c_swcm.alloc(Rp);
        t_.c_bnorm.alloc(Rp); t_.c_rnorm2.alloc(Rp); t_.c_rr.alloc(Rp); t_.c_rr_stop.alloc(Rp);
        t_.c_cg_a.alloc(Rp); t_.c_cg_b.alloc(Rp);
        t_.c_seed.alloc(Rp); t_.c_done.alloc(Rp); t_.c_inner_done.alloc(Rp); t_.c_cg_first.alloc(Rp);
        t_.c_sw.alloc(Rp); t_.c_applied.alloc(Rp); t_.c_flags.alloc(Rp); t_.c_zres.alloc(Rp);
        t_.c_inner_count.alloc(Rp); t_.c_iters.alloc(Rp); t_.c_shift_iters.alloc(Rp);
        t_.c_inner_total.alloc(Rp);
        t_.c_wres.alloc(Rp);
        t_.cg_ha.alloc(Rp * kHist);
        t_.cg_hb.alloc(Rp * kHist);
        const size_t KR = static_cast<size_t>(td.K) * Rp;
        t_.s_pi.alloc(KR); t_.s_pi_prev.alloc(KR); t_.s_pi_next.alloc(KR); t_.s_omega.alloc(KR);
        t_.s_res.alloc(KR); t_.s_last.alloc(KR);
        t_.s_ra.alloc(KR * td.m); t_.s_rb.alloc(KR * td.m); t_.s_rc.alloc(KR * td.m);
        const size_t G = std::max(td.G, td.Gs);
        t_.part_c.alloc(G * Rp);
        t_.part_d.alloc(G * Rp);
        if (full_) {
            t_.ldk = static_cast<size_t>(td.R) * td.N;
            t_.P.alloc(t_.ldk * td.K);
            const bool direct = std::is_same<T, double>::value && req_.G_cols != nullptr &&
                                req_.out_mem == GSC_MEM_DEVICE;
            if (direct) {
                t_.X = reinterpret_cast<cpx<T> *>(req_.G_cols) + static_cast<size_t>(r0_) * td.N;
                ldk_x_ = static_cast<size_t>(req_.R) * td.N;
            } else {
                t_.Xown.alloc(t_.ldk * td.K);
                t_.X = t_.Xown.get();
                ldk_x_ = t_.ldk;
            }
        }
        if (req_.proj != nullptr) {
            const ProjSpec &ps = *req_.proj;
            t_.Mu = ps.M;
            t_.srow = (ps.srow && drhs_ != nullptr) ? 1 : 0;
            const int M = t_.Mu + t_.srow;
            t_.h.alloc(KR * M);
            if (req_.vjp) {
                t_.dh.alloc(KR * M);
                t_.s_dpi.alloc(KR); t_.s_dpi_prev.alloc(KR); t_.s_dpi_next.alloc(KR); t_.s_domega.alloc(KR);
                t_.s_rda.alloc(KR * td.m); t_.s_rdb.alloc(KR * td.m); t_.s_rdc.alloc(KR * td.m);
            } else {
                t_.gacc.alloc(KR * M);
            }
            if (t_.Mu > 0) {
                std::vector<int32_t> idx(static_cast<size_t>(td.Rp) * t_.Mu, 0);
                for (int c = 0; c < td.R; ++c)
                    for (int mm = 0; mm < t_.Mu; ++mm)
                        idx[static_cast<size_t>(c) * t_.Mu + mm] =
                            ps.idx[static_cast<size_t>(r0_ + c) * t_.Mu + mm];
                t_.pidx.alloc(idx.size());
                GSC_HIP(hipMemcpyAsync(t_.pidx.get(), idx.data(), idx.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, st_));
            }
        }
    }

    // Runs the whole iteration; returns the number of outer iterations.
    // Everything before the first outer iteration: state, r = b, the first
    // inner solve by CG (its coefficients give the Chebyshev interval),
    // rho and p.  Synchronises the stream.
    void init_phase(const gsc_opts &o, double inner_tol, int seed0) {
        auto &td = t_.td;
        ColState cs = t_.cols();
        ShiftState ss = t_.shifts(dz_);
        const dim3 eg(td.Rp / 64, td.G), eb(kBlock);
        const int cb = div_up(td.Rp, 256);
        const size_t NR = static_cast<size_t>(td.N) * td.Rp;
        k_init_cols<<<cb, 256, 0, st_>>>(td.R, td.Rp, seed0, cs);
        k_init_shifts<<<div_up(static_cast<int64_t>(td.K) * td.Rp, 256), 256, 0, st_>>>(td.K, td.R, td.Rp, ss);
        if (t_.h.get()) GSC_HIP(hipMemsetAsync(t_.h.get(), 0, t_.h.n * sizeof(c128), st_));
        if (t_.gacc.get()) GSC_HIP(hipMemsetAsync(t_.gacc.get(), 0, t_.gacc.n * sizeof(c128), st_));
        if (t_.dh.get()) GSC_HIP(hipMemsetAsync(t_.dh.get(), 0, t_.dh.n * sizeof(c128), st_));
        GSC_HIP(hipGetLastError());
        // r = b, r'_0 = S^{-1} b, p = r'_0, rho = r'^T r
        k_init_rhs<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, td.R, drhs_, dB_, t_.r.get(), t_.res.get(),
                                         t_.d.get(), t_.part_d.get());
        k_col_rnorm<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, t_.part_d.get(), 1, inner_tol, cs);
        if (full_)
            k_zero_done_cols<T><<<dim3(div_up(td.N, 256), std::min(td.R, 1024)), 256, 0, st_>>>(
                td.K, td.R, td.N, ldk_x_, t_.c_done.get(), t_.X);
        inner_tol_ = inner_tol;
        inner_tol_base_ = inner_tol;
        inner_solve_cg(o, cs, t_.ring.get());
        if (full_) {
            k_ring_transpose<T><<<dim3(td.Rp / 64, std::min(div_up(td.N, 32), 65535)), kBlock, 0, st_>>>(td.N, td.Rp, t_.ring.get(),
                                                                                      t_.ringT.get());
        }
        if (o.inner_method != 1) setup_chebyshev(o, inner_tol);
        k_rho_dot<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_done.get(), t_.c_zres.get(), t_.ring.get(),
                                        t_.r.get(), t_.part_c.get());
        k_init_rho<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, t_.part_c.get(), cs);
        k_p_update<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, 1, cs, t_.ring.get(), t_.r.get(), t_.p.get(),
                                         t_.P.get(), t_.ldk, nullptr);
        GSC_HIP(hipGetLastError());
        check_status(false);
        (void)NR;
    }

    // One outer iteration of a projected-carry tile with no host
    // synchronisation (graph-capturable: the kernels do not depend on n
    // beyond the profiling histogram).
    void enqueue_projected_iteration(const gsc_opts &o, int n) {
        auto &td = t_.td;
        ColState cs = t_.cols();
        ShiftState ss = t_.shifts(dz_);
        const dim3 eg(td.Rp / 64, td.G), eb(kBlock);
        const T *Sv = sval(), *Hv = hval();
        cpx<T> *rp = t_.ring.get();   // m = 1 for the projected carry
        launch_spmm_seed<T>(st_, pr_, td, Sv, Hv, t_.p.get(), t_.q.get(), dz_, t_.c_seed.get(), t_.c_done.get(),
                            t_.part_c.get());
        k_ctrl<<<td.Rp, kBlock, 0, st_>>>(td.K, td.Rp, td.Gs, n, 0, t_.part_c.get(), cs, ss);
        proj_update(cs, ss, 0, rp);
        k_update_r<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_done.get(), t_.c_alpha.get(), t_.q.get(),
                                         t_.r.get(), t_.res.get(), t_.d.get(), t_.part_d.get(), cheb_ok_ ? 0 : 1,
                                         r32_out());
        k_col_rnorm<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, t_.part_d.get(), 0, inner_tol_, cs);
        const bool fused = inner_solve(o, cs, rp, t_.part_c.get());
        if (!fused)
            k_rho_dot<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_done.get(), t_.c_zres.get(), rp, t_.r.get(),
                                            t_.part_c.get());
        k_post<<<td.Rp, kBlock, 0, st_>>>(td.K, td.Rp, fused ? td.Gs : td.G, n, 0, t_.part_c.get(), o.tol, cs, ss,
                                          t_.h.get(), t_.dh.get(), t_.Mu + t_.srow);
        k_p_update<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, 0, cs, rp, t_.r.get(), t_.p.get(), t_.P.get(),
                                         t_.ldk, nullptr);
        GSC_HIP(hipGetLastError());
    }

    bool chebyshev_ready() const { return cheb_ok_; }
    hipStream_t stream() const { return st_; }
    void set_stream(hipStream_t s) { st_ = s; }
    // enqueue the status reduction and its copy into host memory `h`
    void enqueue_status(Status *d, Status *h) {
        k_status<<<1, kBlock, 0, st_>>>(t_.td.Rp, t_.cols(), d);
        GSC_HIP(hipGetLastError());
        GSC_HIP(hipMemcpyAsync(h, d, sizeof(Status), hipMemcpyDeviceToHost, st_));
    }
    // relaxed inner tolerance from a polled status (see relax_inner)
    bool relax_from_status(const Status &s, bool steps_only) { return relax_inner(s.worst_res, steps_only); }
    void note_status(const Status &s) {
        flags_ |= s.flags;
        if (s.flags & FLAG_NAN) throw Error(GSC_E_NAN, "non-finite value in the iteration");
        if (s.flags & FLAG_NOT_SPD) throw Error(GSC_E_S_NOT_SPD, "inner CG found d^H S d <= 0: S is not positive definite");
        if (s.flags & FLAG_BREAKDOWN) throw Error(GSC_E_BREAKDOWN, "COCG breakdown (p^T A p or r'^T r vanished)");
    }

    int run(const gsc_opts &o, double inner_tol, int seed0) {
        init_phase(o, inner_tol, seed0);
        auto &td = t_.td;
        ColState cs = t_.cols();
        ShiftState ss = t_.shifts(dz_);
        const dim3 eg(td.Rp / 64, td.G), eb(kBlock);
        const int cb = div_up(td.Rp, 256);
        const size_t NR = static_cast<size_t>(td.N) * td.Rp;
        const T *Sv = sval(), *Hv = hval();
        int n0 = 0;   // first unflushed step (full carry)
        int n = 0;
        for (; n < o.max_iter; ++n) {
            const int slot = n % td.m, slot_next = (n + 1) % td.m;
            cpx<T> *rp_n = t_.ring.get() + slot * NR;
            cpx<T> *rp_next = t_.ring.get() + slot_next * NR;
            prof_.begin(st_, KP_SPMM_SEED, 2.0 * mat_bytes());
            launch_spmm_seed<T>(st_, pr_, td, Sv, Hv, t_.p.get(), t_.q.get(), dz_, t_.c_seed.get(),
                                t_.c_done.get(), t_.part_c.get());
            prof_.end(st_);
            prof_.begin(st_, KP_CTRL, 0.0);
            k_ctrl<<<td.Rp, kBlock, 0, st_>>>(td.K, td.Rp, td.Gs, n, slot, t_.part_c.get(), cs, ss);
            prof_.end(st_);
            if (full_) {
                if (n + 1 - n0 == td.m) {
                    flush(cs, ss, n0, n + 1, 0);
                    n0 = n + 1;
                }
            } else {
                proj_update(cs, ss, slot, rp_n);
            }
            prof_.begin(st_, KP_UPDATE_R, 0.0);
            k_update_r<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_done.get(), t_.c_alpha.get(),
                                             t_.q.get(), t_.r.get(), t_.res.get(), t_.d.get(), t_.part_d.get(),
                                             cheb_ok_ ? 0 : 1, r32_out());
            prof_.end(st_);
            k_col_rnorm<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, t_.part_d.get(), 0, inner_tol, cs);
            // rho = r'^T r comes out of the Chebyshev iteration's last step
            // (partials over its row groups), else from its own pass
            const bool fused = inner_solve(o, cs, rp_next, t_.part_c.get());
            if (!fused) {
                prof_.begin(st_, KP_RHO_DOT, 0.0);
                k_rho_dot<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_done.get(), t_.c_zres.get(), rp_next,
                                                t_.r.get(), t_.part_c.get());
                prof_.end(st_);
            }
            prof_.begin(st_, KP_POST, 0.0);
            k_post<<<td.Rp, kBlock, 0, st_>>>(td.K, td.Rp, fused ? td.Gs : td.G, n, full_ ? 1 : 0, t_.part_c.get(),
                                              o.tol, cs, ss, t_.h.get(), t_.dh.get(), t_.Mu + t_.srow);
            prof_.end(st_);
            GSC_HIP(hipGetLastError());
            const Status s = check_status(true);
            if (o.inner_relax) relax_inner(s.worst_res);
            if (full_ && s.switched > 0) {
                flush(cs, ss, n0, n + 1, 1, s.switched);
                k_mark_applied<<<cb, 256, 0, st_>>>(td.Rp, n + 1, cs);
            }
            // the seed update also writes the column-major copy of r' (after
            // its switch rescale) when one block's row tile fits LDS
            const bool fuse_t = full_ && td.Lr <= 64;
            const size_t tshm = fuse_t ? 64 * static_cast<size_t>(td.Lr + 1) * sizeof(cpx<T>) : 0;
            prof_.begin(st_, KP_P_UPDATE, 0.0);
            k_p_update<T><<<eg, eb, tshm, st_>>>(td.N, td.Rp, td.Lr, 0, cs, rp_next, t_.r.get(), t_.p.get(),
                                                t_.P.get(), t_.ldk,
                                                fuse_t ? t_.ringT.get() + slot_next * NR : nullptr);
            prof_.end(st_);
            if (full_ && !fuse_t) {
                prof_.begin(st_, KP_RING_T, 0.0);
                k_ring_transpose<T><<<dim3(td.Rp / 64, std::min(div_up(td.N, 32), 65535)), kBlock, 0, st_>>>(
                    td.N, td.Rp, rp_next, t_.ringT.get() + slot_next * NR);
                prof_.end(st_);
            }
            if (s.active_cols == 0) { ++n; break; }
        }
        if (full_ && n > n0) flush(cs, ss, n0, n, 0);
        GSC_HIP(hipGetLastError());
        if (prof_.on) account_bytes(n);
        return n;
    }


    // Generalised Lanczos (Sec. 3.2) for the P processes of this tile (two per
    // column).  Device outputs: a, b [2Rp][mmax] (zeroed here; b[p][0] = 0),
    // steps, vj [2Rp], G [K][ldo] at column offset p0.  Returns the steps run.
    int run_lanczos(const gsc_opts &o, double inner_tol, const int64_t *rhs, int P, int mmax, double tol, int check,
                    double *a, double *b, int *steps, double *vj, c128 *gout, int ldo, int p0) {
        auto &td = t_.td;
        ColState cs = t_.cols();
        const dim3 eg(td.Rp / 64, td.G), eb(kBlock);
        const int cb = div_up(td.Rp, 256);
        const size_t NR = static_cast<size_t>(td.N) * td.Rp;
        const int Gm = std::max(td.G, td.Gs);
        DevBuf<double> part(3 * static_cast<size_t>(Gm) * td.Rp), inv(2 * static_cast<size_t>(td.Rp));
        DevBuf<int> done(2 * static_cast<size_t>(td.Rp));
        DevBuf<c128> gprev(static_cast<size_t>(std::max(P, 1)) * td.K);
        DevBuf<cpx<T>> ub0(NR), ub1(NR), sb0(NR), sb1(NR);
        GSC_HIP(hipMemsetAsync(a, 0, 2 * static_cast<size_t>(td.Rp) * mmax * sizeof(double), st_));
        GSC_HIP(hipMemsetAsync(b, 0, 2 * static_cast<size_t>(td.Rp) * mmax * sizeof(double), st_));
        k_init_cols<<<cb, 256, 0, st_>>>(td.R, td.Rp, 0, cs);
        k_lz_unit<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, P, rhs, t_.r.get(), t_.res.get(), t_.d.get(),
                                         part.get());
        k_col_rnorm<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, part.get(), 1, inner_tol, cs);
        inner_tol_ = inner_tol;
        cpx<T> *v = t_.ring.get();   // S^{-1} e_j, then the inner solve's output w
        inner_solve_cg(o, cs, v);
        if (o.inner_method != 1) setup_chebyshev(o, inner_tol);
        cpx<T> *u = ub0.get(), *up = ub1.get(), *s = sb0.get(), *sp = sb1.get();
        k_lz_vj<T><<<div_up(2 * td.Rp, 256), 256, 0, st_>>>(P, td.Rp, rhs, v, vj, inv.get(), steps, done.get());
        k_lz_start<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, inv.get(), v, u, up, sp);
        k_lz_fill<<<div_up(gprev.n, 256), 256, 0, st_>>>(gprev.n, c128{1e300, 0.0}, gprev.get());
        k_lz_cols<<<cb, 256, 0, st_>>>(td.Rp, done.get(), cs.done);
        GSC_HIP(hipGetLastError());
        check_status(false);
        const T *Hv = hval(), *Sv = sval();
        const size_t Gs = static_cast<size_t>(td.Gs);
        int ran = 0;
        for (int n = 0; n < mmax; ++n) {
            prof_.begin(st_, KP_LZ_HPROD, 2.0 * mat_bytes() + 3.0 * last_active_ * td.N * sizeof(cpx<T>));
            launch_lz_hprod<T>(st_, pr_, td, Hv, Sv, u, t_.r.get(), s, cs.done, part.get());
            prof_.end(st_);
            k_lz_reduce_a<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, part.get(), n, mmax, a, steps, done.get());
            ran = n + 1;
            if (n == mmax - 1) break;
            k_col_rnorm<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, part.get() + 2 * Gs * td.Rp, 0, inner_tol, cs);
            if (!cheb_ok_) {
                k_copy_vec<T><<<div_up(NR, 256), 256, 0, st_>>>(NR, t_.r.get(), t_.res.get());
                k_copy_vec<T><<<div_up(NR, 256), 256, 0, st_>>>(NR, t_.r.get(), t_.d.get());
            }
            inner_solve(o, cs, v);
            prof_.begin(st_, KP_LZ_UPDATE, 7.0 * last_active_ * td.N * sizeof(cpx<T>));
            k_lz_update<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, td.G, n, mmax, a, b, v, u, up, t_.r.get(), s, sp,
                                               part.get());
            prof_.end(st_);
            k_lz_reduce_b<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, part.get(), n, mmax, a, b, inv.get(), done.get());
            prof_.begin(st_, KP_LZ_SCALE, 2.0 * last_active_ * td.N * sizeof(cpx<T>));
            k_lz_scale<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, inv.get(), v, up);
            prof_.end(st_);
            std::swap(u, up);
            std::swap(s, sp);
            GSC_HIP(hipGetLastError());
            if (check > 0 && (n + 1) % check == 0) {
                k_lz_cf<<<P, kBlock, 0, st_>>>(td.K, mmax, dz_, a, b, vj, steps, gprev.get(), tol, done.get(), 0,
                                               nullptr, 0, 0);
                k_lz_cols<<<cb, 256, 0, st_>>>(td.Rp, done.get(), cs.done);
                const Status st = check_status(false);
                if (st.active_cols == 0) break;
            }
        }
        k_lz_cf<<<P, kBlock, 0, st_>>>(td.K, mmax, dz_, a, b, vj, steps, gprev.get(), tol, done.get(), 1, gout, ldo,
                                       p0);
        GSC_HIP(hipGetLastError());
        lz_steps_ = ran;
        return ran;
    }

    int flags() const { return flags_; }

    void write_outputs(gsc_stats *stats, double *res_host, unsigned char *conv_host, double tol, int nrhs_total) {
        auto &td = t_.td;
        (void)stats;
        if (full_) {
            if (req_.G_cols != nullptr && t_.X == t_.Xown.get()) {
                if (req_.out_mem == GSC_MEM_DEVICE) {
                    const int64_t tot = static_cast<int64_t>(td.R) * td.N * td.K;
                    k_store_cols<T><<<div_up(tot, 256), 256, 0, st_>>>(
                        td.K, td.R, td.N, t_.X, ldk_x_, reinterpret_cast<c128 *>(req_.G_cols), nrhs_total, r0_);
                } else {
                    // widen on the device, then copy each shift's slab
                    DevBuf<c128> tmp(static_cast<size_t>(td.R) * td.N * td.K);
                    const int64_t tot = static_cast<int64_t>(td.R) * td.N * td.K;
                    k_store_cols<T><<<div_up(tot, 256), 256, 0, st_>>>(td.K, td.R, td.N, t_.X, ldk_x_, tmp.get(),
                                                                      td.R, 0);
                    GSC_HIP(hipGetLastError());
                    const size_t slab = static_cast<size_t>(td.R) * td.N * sizeof(c128);
                    if (td.R == nrhs_total) {
                        // one tile: the whole [K][R][N] block is contiguous on both sides
                        copy_to_host(req_.G_cols, tmp.get(), slab * td.K, st_);
                    } else {
                        for (int k = 0; k < td.K; ++k)
                            copy_to_host(req_.G_cols + 2 * ((static_cast<size_t>(k) * nrhs_total + r0_) * td.N),
                                         tmp.get() + static_cast<size_t>(k) * td.R * td.N, slab, st_);
                    }
                }
            }
            if (req_.G_proj != nullptr && req_.nproj > 0) {
                std::vector<int32_t> idx(static_cast<size_t>(td.R) * req_.nproj);
                for (int c = 0; c < td.R; ++c)
                    for (int mm = 0; mm < req_.nproj; ++mm)
                        idx[static_cast<size_t>(c) * req_.nproj + mm] =
                            static_cast<int32_t>(req_.proj_idx[static_cast<size_t>(r0_ + c) * req_.nproj + mm]);
                DevBuf<int32_t> didx(idx.size());
                GSC_HIP(hipMemcpyAsync(didx.get(), idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                       st_));
                const int64_t tot = static_cast<int64_t>(td.K) * td.R * req_.nproj;
                if (req_.out_mem == GSC_MEM_DEVICE) {
                    k_gather_proj<T><<<div_up(tot, 256), 256, 0, st_>>>(td.K, td.R, td.N, req_.nproj, didx.get(),
                                                                       t_.X, ldk_x_,
                                                                       reinterpret_cast<c128 *>(req_.G_proj),
                                                                       nrhs_total, r0_);
                    GSC_HIP(hipStreamSynchronize(st_));
                } else {
                    DevBuf<c128> tmp(static_cast<size_t>(td.K) * td.R * req_.nproj);
                    k_gather_proj<T><<<div_up(tot, 256), 256, 0, st_>>>(td.K, td.R, td.N, req_.nproj, didx.get(),
                                                                       t_.X, ldk_x_, tmp.get(), td.R, 0);
                    std::vector<c128> h(tmp.n);
                    GSC_HIP(hipMemcpyAsync(h.data(), tmp.get(), h.size() * sizeof(c128), hipMemcpyDeviceToHost,
                                           st_));
                    GSC_HIP(hipStreamSynchronize(st_));
                    for (int k = 0; k < td.K; ++k)
                        for (int c = 0; c < td.R; ++c)
                            std::memcpy(req_.G_proj + 2 * ((static_cast<size_t>(k) * nrhs_total + r0_ + c) * req_.nproj),
                                        h.data() + (static_cast<size_t>(k) * td.R + c) * req_.nproj,
                                        req_.nproj * sizeof(c128));
                }
                GSC_HIP(hipGetLastError());
            }
            if (req_.sg_diag != nullptr) {
                const int64_t tot = static_cast<int64_t>(td.K) * td.R;
                k_sx_diag<T><<<div_up(tot, 256), 256, 0, st_>>>(td.K, td.R, td.N, td.B, pr_.rowptr.get(),
                                                               pr_.colidx.get(), pr_.S.get(), drhs_, t_.X, ldk_x_,
                                                               req_.sg_diag, nrhs_total, r0_);
                GSC_HIP(hipGetLastError());
            }
        } else if (req_.proj_out != nullptr && t_.gacc.get() != nullptr) {
            const int M = t_.Mu + t_.srow;
            const int64_t tot = static_cast<int64_t>(td.K) * td.R * M;
            k_store_proj<<<div_up(tot, 256), 256, 0, st_>>>(td.K, td.R, td.Rp, M, t_.gacc.get(), req_.proj_out,
                                                            nrhs_total, r0_);
            GSC_HIP(hipGetLastError());
        }
        // per (k, r) residual estimates
        std::vector<double> res(static_cast<size_t>(td.K) * td.Rp);
        GSC_HIP(hipMemcpyAsync(res.data(), t_.s_res.get(), res.size() * sizeof(double), hipMemcpyDeviceToHost, st_));
        std::vector<long long> si(td.Rp);
        std::vector<int> inner(td.Rp), iters(td.Rp);
        GSC_HIP(hipMemcpyAsync(si.data(), t_.c_shift_iters.get(), si.size() * sizeof(long long),
                               hipMemcpyDeviceToHost, st_));
        GSC_HIP(hipStreamSynchronize(st_));
        for (int k = 0; k < td.K; ++k)
            for (int c = 0; c < td.R; ++c) {
                const double v = res[static_cast<size_t>(k) * td.Rp + c];
                if (res_host) res_host[static_cast<size_t>(k) * nrhs_total + r0_ + c] = v;
                if (conv_host) conv_host[static_cast<size_t>(k) * nrhs_total + r0_ + c] = v <= tol ? 1 : 0;
                worst_res_ = std::max(worst_res_, v);
            }
        for (int c = 0; c < td.R; ++c) shift_rhs_iters_ += si[c];
    }

    void true_residual(double *out_host, int nrhs_total) {
        auto &td = t_.td;
        DevBuf<double> out(static_cast<size_t>(td.K) * td.R);
        dim3 grid(td.R, td.K);
        k_true_residual<T><<<grid, kBlock, 0, st_>>>(td.K, td.R, td.N, td.B, pr_.rowptr.get(), pr_.colidx.get(),
                                                    pr_.S.get(), pr_.H.get(), dz_, drhs_, dB_, t_.X, ldk_x_,
                                                    out.get());
        GSC_HIP(hipGetLastError());
        std::vector<double> h(out.n);
        GSC_HIP(hipMemcpyAsync(h.data(), out.get(), h.size() * sizeof(double), hipMemcpyDeviceToHost, st_));
        GSC_HIP(hipStreamSynchronize(st_));
        for (int k = 0; k < td.K; ++k)
            for (int c = 0; c < td.R; ++c)
                out_host[static_cast<size_t>(k) * nrhs_total + r0_ + c] = h[static_cast<size_t>(k) * td.R + c];
    }

    long long inner_total() const { return inner_total_; }
    // graph replays run no host code: the scheduler keeps the count instead
    void set_inner_total(long long v) { inner_total_ = v; }
    int cheb_steps_per_solve() const { return mixed_ ? mx_steps_per_solve() : cheb_steps_ - 1; }

    // Algorithmic bytes of one outer iteration of one column in projected
    // carry with the current inner plan (vectors of N elements read or
    // written once: seed product p, q; r update r, q, r; p update r', p, p;
    // the Chebyshev steps' gathered, streamed and written vectors; plus the
    // matrices once per product launch, shared by the tile's Rp columns).
    // The projections' scalar updates and the column reductions are left
    // out (K M scalars against N-long vectors).
    double col_iter_inner_bytes() const {
        const auto &td = t_.td;
        const double s = sizeof(cpx<T>), N = td.N;
        const double mat = static_cast<double>(pr_.nnzb) * pr_.B * pr_.B;
        double v = 0.0, m = 0.0;
        if (!cheb_ok_) return 0.0;
        if (mixed_) {
            const int nr = static_cast<int>(mx_plan_.size());
            for (int j = 0; j < nr; ++j) {
                const int K = mx_plan_[j];
                for (int kk = 1; kk < K; ++kk) {
                    const int mode = kk == 1 ? 0 : kk == 2 ? 1 : 2;
                    const bool last = kk == K - 1;
                    const int fin = last ? (j == 0 ? 1 : 2) : 0;
                    v += 8.0 + (mode >= 1 ? 8.0 : 0.0) + (mode == 2 ? 8.0 : 0.0);
                    v += fin == 0 ? 8.0 : fin == 1 ? 16.0 : 32.0;
                    if (last && j == nr - 1) v += 16.0;   // r for the dot
                    m += 4.0 * mat;
                }
                if (j > 0) { v += 40.0; m += 8.0 * mat; }
            }
        } else {
            for (int k = 1; k < cheb_steps_; ++k) {
                v += s * (k == 1 ? 2 : k == 2 ? 3 : 4);
                m += sizeof(T) * mat;
            }
        }
        return v * N + m / td.Rp;
    }
    double col_iter_bytes() const {
        const auto &td = t_.td;
        const double s = sizeof(cpx<T>), N = td.N;
        const double mat = static_cast<double>(pr_.nnzb) * pr_.B * pr_.B;
        const double outer = (2.0 + 3.0 + 3.0) * s * N + (mixed_ ? 8.0 * N : 0.0) + 2.0 * sizeof(T) * mat / td.Rp;
        return outer + col_iter_inner_bytes();
    }
    int switches() const { return switches_; }
    long long shift_rhs_iters() const { return shift_rhs_iters_; }
    double worst_res() const { return worst_res_; }

  private:
    const T *sval() const;
    const T *hval() const;

    // Algorithmic bytes of every kernel class over this solve (the method's
    // own reads and writes of N-long vectors; gathers and re-reads excluded),
    // from per-column iteration counters and the per-iteration active counts.
    void account_bytes(int n_iters) {
        auto &td = t_.td;
        std::vector<int> it(td.Rp);
        std::vector<long long> act(std::max(1, n_iters)), cols(std::max(1, n_iters));
        GSC_HIP(hipMemcpyAsync(it.data(), t_.c_iters.get(), td.Rp * sizeof(int), hipMemcpyDeviceToHost, st_));
        if (n_iters > 0) {
            GSC_HIP(hipMemcpyAsync(act.data(), t_.act_hist.get(), n_iters * sizeof(long long),
                                   hipMemcpyDeviceToHost, st_));
            GSC_HIP(hipMemcpyAsync(cols.data(), t_.col_hist.get(), n_iters * sizeof(long long),
                                   hipMemcpyDeviceToHost, st_));
        }
        GSC_HIP(hipStreamSynchronize(st_));
        double s_it = 0;
        for (int c = 0; c < td.R; ++c) s_it += it[c];
        const double solves = s_it + td.R;
        const double vec = static_cast<double>(td.N) * sizeof(cpx<T>);
        prof_.add_bytes(KP_SPMM_SEED, s_it * vec * 2);
        prof_.add_bytes(KP_UPDATE_R, s_it * vec * (cheb_ok_ ? 3 : 5));
        prof_.add_bytes(KP_RHO_DOT, solves * vec * 2);
        const bool fused_t = full_ && td.Lr <= 64;
        prof_.add_bytes(KP_P_UPDATE, solves * vec * (fused_t ? 4 : 3));
        if (full_ && !fused_t) prof_.add_bytes(KP_RING_T, solves * vec * 2);
        double fb = 0;
        for (const auto &f : flushes_) {
            const int n0 = f[0], n1 = f[1], nsw = f[2];
            if (n0 >= n_iters) continue;
            const double a = static_cast<double>(act[n0]), cc = static_cast<double>(cols[n0]);
            if (nsw < 0) {
                fb += (4.0 * a + cc * (n1 - n0)) * vec;        // full pass over every active (k, c)
            } else if (cc > 0) {
                fb += nsw * (4.0 * a / cc + (n1 - n0)) * vec;  // seed-switch columns only
            }
        }
        prof_.add_bytes(KP_SHIFT_UPDATE, fb);
        prof_.resolve();
    }
    std::vector<std::array<int, 3>> flushes_;
    double mat_bytes() const { return static_cast<double>(pr_.nnzb) * pr_.B * pr_.B * sizeof(T); }

    Status check_status(bool count_switch) {
        auto &td = t_.td;
        k_status<<<1, kBlock, 0, st_>>>(td.Rp, t_.cols(), hs_.hd);
        GSC_HIP(hipGetLastError());
        GSC_HIP(hipStreamSynchronize(st_));
        const Status s = *hs_.h;
        flags_ |= s.flags;
        last_active_ = s.active_cols;
        if (count_switch) switches_ += s.switched;
        if (s.flags & FLAG_NAN) throw Error(GSC_E_NAN, "non-finite value in the iteration");
        if (s.flags & FLAG_NOT_SPD) throw Error(GSC_E_S_NOT_SPD, "inner CG found d^H S d <= 0: S is not positive definite");
        if (s.flags & FLAG_BREAKDOWN) throw Error(GSC_E_BREAKDOWN, "COCG breakdown (p^T A p or r'^T r vanished)");
        return s;
    }

    // S y = r; with dot_part, returns true when the partials of y^T r over
    // the product kernels' row groups (td.Gs) were left there as well
    bool inner_solve(const gsc_opts &o, ColState cs, cpx<T> *y, c128 *dot_part = nullptr) {
        if (cheb_ok_ && mixed_) return inner_solve_mx(cs, reinterpret_cast<c128 *>(y), dot_part);
        if (cheb_ok_) return inner_solve_cheb(o, cs, y, dot_part);
        inner_solve_cg(o, cs, y);
        return false;
    }

    // Interval for the Chebyshev iteration from the Ritz values of the first
    // (CG) inner solve over all columns, widened by 10 % of its width.
    void setup_chebyshev(const gsc_opts &o, double tol_in) {
        auto &td = t_.td;
        DevBuf<double> lmin(td.Rp), lmax(td.Rp), out(2);
        ColState cs = t_.cols();
        k_ritz<<<div_up(td.Rp, 64), 64, 0, st_>>>(td.R, td.Rp, cs, lmin.get(), lmax.get());
        k_ritz_reduce<<<1, kBlock, 0, st_>>>(td.Rp, lmin.get(), lmax.get(), out.get());
        GSC_HIP(hipGetLastError());
        double h[2];
        GSC_HIP(hipMemcpyAsync(h, out.get(), sizeof(h), hipMemcpyDeviceToHost, st_));
        GSC_HIP(hipStreamSynchronize(st_));
        cheb_ok_ = false;
        if (!(h[0] < 1e299 && h[1] > -1e299)) return;
        const double w = h[1] - h[0];
        const double pad = std::max(0.1 * w, 1e-3 * std::fabs(h[1]));
        const double a = h[0] - pad, b = h[1] + pad;
        if (!(a > 0.0) || !std::isfinite(b)) return;
        cheb_theta_ = 0.5 * (b + a);
        cheb_delta_ = 0.5 * (b - a);
        const double kappa = b / a;
        cheb_rho_ = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
        cheb_max_ = o.inner_max_iter;
        cheb_steps_ = cheb_steps_for(tol_in);
        if (mixed_) mx_plan_ = mx_plan_for(tol_in);
        cheb_ok_ = true;
        cheb_lo_ = h[0];
        cheb_hi_ = h[1];
    }

    // steps K of the Chebyshev iteration for a relative residual tol: the
    // error bound 2 rho^K of the interval
    int cheb_steps_for(double tol) const {
        const double lr = std::log(1.0 / std::max(cheb_rho_, 1e-300));
        const int k = std::max(2, static_cast<int>(std::ceil(std::log(2.0 / tol) / lr)));
        return std::min(k, cheb_max_);
    }

    // Relaxed inner tolerance (option inner_relax).  An error e in r' = S^-1 r
    // enters shift k's iterate as e / pi^k, i.e. scaled by that shift's
    // residual ||r|| / (|pi^k| ||b||); a relative inner tolerance of
    // tol_in / (largest residual still above tol) therefore keeps what every
    // unconverged shift receives at tol_in relative to ||b||, as in its first
    // iteration.  Capped at kRelaxCap; the fixed tolerance is the floor.
    // With steps_only, the tolerance changes only together with the step
    // count (a captured graph holds both); returns whether the count changed.
    bool relax_inner(double worst, bool steps_only = false) {
        if (!cheb_ok_ || !(inner_tol_base_ > 0.0)) return false;
        double t = worst > 0.0 ? inner_tol_base_ / worst : inner_tol_base_;
        t = std::max(std::min(t, kRelaxCap), inner_tol_base_);
        bool changed;
        if (mixed_) {
            std::vector<int> plan = mx_plan_for(t);
            changed = plan != mx_plan_;
            mx_plan_ = std::move(plan);
        } else {
            const int k = cheb_steps_for(t);
            changed = k != cheb_steps_;
            cheb_steps_ = k;
        }
        if (changed || !steps_only) inner_tol_ = t;
        return changed;
    }

    // Rounds of the mixed inner solve for a relative tolerance tau: one
    // round when tau >= kMxSingle (a few times what the FP32 residual
    // estimate resolves), else rounds asked for kMxFloor each, the FP64
    // residual between rounds carrying the rest.  A round of K steps
    // reaches its Chebyshev bound 2 rho^K, but no lower than kMxReach, where
    // complex64 arithmetic stagnates: the next round is planned for what is
    // left after that (the residual check after the last round catches a
    // round that fell short).  Entries are the step counts K_j.
    std::vector<int> mx_plan_for(double tau) const {
        std::vector<int> plan;
        // down to kMxSingle one complex64 round is cheaper than two rounds
        // and an FP64 residual pass
        if (tau >= kMxSingle) return {cheb_steps_for(tau)};
        double rem = tau;
        while (true) {
            const int k = cheb_steps_for(std::max(rem, kMxFloor));
            plan.push_back(k);
            if (rem >= kMxFloor * (1.0 - 1e-9) || plan.size() == 4) break;
            rem /= std::max(2.0 * std::pow(cheb_rho_, k), kMxReach);
        }
        return plan;
    }

    // Mixed inner solve of S Y = r (Y complex128, the ring slot): rounds of
    // the complex64 Chebyshev iteration (FP32 S and arithmetic, iterates in
    // complex64) refined in FP64: round 1 solves S y = r, round j > 1 solves
    // S y = r - S Y for the FP64 residual of the sum so far, and every round
    // adds its last iterate to Y in FP64 (iterative refinement).  The last
    // step of the last round also forms the partials of Y^T r (the next rho)
    // when dot_part is given.  Then the residual check of the Chebyshev
    // path: columns whose last round ended above tol / rho take one more
    // refinement round, and a final check flags those still above tol.  No
    // host synchronisation (graph-capturable); the plan comes from the
    // current inner tolerance.
    bool inner_solve_mx(ColState cs, c128 *Y, c128 *dot_part) {
        if constexpr (!std::is_same<T, double>::value) {
            (void)cs; (void)Y; (void)dot_part;
            throw Error(GSC_E_ARG, "the mixed inner solve runs on the FP64 seed process");
        } else {
        auto &td = t_.td;
        const size_t NR = static_cast<size_t>(td.N) * td.Rp;
        if (!r32_fresh_) {
            k_to_c64<<<div_up(static_cast<int64_t>(NR), 256), 256, 0, st_>>>(NR, t_.r.get(), mx_f_.get());
            GSC_HIP(hipGetLastError());
        }
        r32_fresh_ = false;
        const bool dot = dot_part != nullptr;
        const float *S32 = pr_.S32.get();
        const double *S64 = pr_.S.get();
        const double sigma = cheb_theta_ / cheb_delta_;
        c64 *buf[2] = {mx_ya_.get(), mx_yb_.get()};
        const int cb = td.cb > 0 ? td.cb : td.Rp;
        const double vec = static_cast<double>(last_active_) * td.N;
        // one complex64 round of K - 1 steps on S y = f (f in mx_f_)
        auto round = [&](int K, int fin, bool with_dot, const int *skip, int c0, int w, int dot_active_only,
                         double cols, bool timed) {
            double rho_prev = 1.0 / sigma, bytes = 0.0;
            if (timed) prof_.begin_group(st_, KP_CHEB_MX);
            for (int kk = 1; kk < K; ++kk) {
                const double rho = 1.0 / (2.0 * sigma - rho_prev);
                const double c1 = rho * rho_prev, c2 = 2.0 * rho / cheb_delta_;
                const int mode = kk == 1 ? 0 : kk == 2 ? 1 : 2;
                const bool last = kk == K - 1;
                const int f = last ? fin : 0;
                launch_cheb_mx(st_, pr_, td, mode, f, last && with_dot, c0, w, S32, buf[kk % 2], mx_f_.get(),
                               buf[(kk + 1) % 2], Y, t_.r.get(), skip, 1.0 / cheb_theta_, c1, c2, t_.part_d.get(),
                               dot_part, dot_active_only);
                // algorithmic bytes per column element: gathered y (or f),
                // f and y_{k-1} streamed, y_{k+1} written; a final step writes
                // Y (complex128, after reading it for fin 2) and reads r for
                // the dot
                double b = 8.0 + (mode >= 1 ? 8.0 : 0.0) + (mode == 2 ? 8.0 : 0.0);
                b += f == 0 ? 8.0 : f == 1 ? 16.0 : 32.0;
                if (last && with_dot) b += 16.0;
                bytes += b * cols * td.N;
                rho_prev = rho;
            }
            if (timed) prof_.end_group(st_, K - 1, bytes);
        };
        const int nr = static_cast<int>(mx_plan_.size());
        const double wfrac = 1.0 / td.Rp;
        for (int c0 = 0; c0 < td.Rp; c0 += cb) {
            const int w = std::min(cb, td.Rp - c0);
            const double cols = vec / td.N * w * wfrac;
            for (int j = 0; j < nr; ++j) {
                if (j > 0) {
                    prof_.begin(st_, KP_MX_RESID, 40.0 * cols * td.N);
                    launch_mx_resid(st_, pr_, td, c0, w, S64, Y, t_.r.get(), mx_f_.get(), t_.c_done.get(),
                                    t_.part_d.get());
                    prof_.end(st_);
                }
                round(mx_plan_[j], j == 0 ? 1 : 2, dot && j == nr - 1, t_.c_done.get(), c0, w, 0, cols, true);
            }
        }
        k_cheb_check<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, t_.part_d.get(), inner_tol_ / cheb_rho_, 0, cs);
        // one more refinement round for the columns that failed the check
        // (the launches skip every other column; neither timed nor counted)
        for (int c0 = 0; c0 < td.Rp; c0 += cb) {
            const int w = std::min(cb, td.Rp - c0);
            launch_mx_resid(st_, pr_, td, c0, w, S64, Y, t_.r.get(), mx_f_.get(), t_.c_inner_done.get(),
                            t_.part_d.get());
            round(kMxSafetySteps, 2, dot, t_.c_inner_done.get(), c0, w, 1, 0.0, false);
        }
        k_cheb_check<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, t_.part_d.get(), inner_tol_, 1, cs);
        GSC_HIP(hipGetLastError());
        inner_total_ += mx_steps_per_solve();
        return dot;
        }
    }
    // products with S per mixed inner solve (Chebyshev steps and FP64
    // residual passes), without the safety round
    int mx_steps_per_solve() const {
        int n = 0;
        for (size_t j = 0; j < mx_plan_.size(); ++j) n += mx_plan_[j] - 1 + (j > 0 ? 1 : 0);
        return n;
    }
    c64 *r32_out() {
        if (!mixed_ || !cheb_ok_) return nullptr;
        r32_fresh_ = true;
        return mx_f_.get();
    }

    // Chebyshev iteration for S y = r (r in t_.r), y_K written to `ytarget`,
    // with no host synchronisation: K - 1 fused steps, a residual check of
    // y_{K-1} at tol / rho, two more steps only for the columns that failed
    // it (the parity brings their y_{K+2} back into `ytarget`), and a final
    // check at tol that flags columns still above it.  Three-term form:
    // step k reads y_k (gathered) and y_{k-1} and writes y_{k+1} over y_{k-1},
    // so two buffers alternate.
    bool inner_solve_cheb(const gsc_opts &o, ColState cs, cpx<T> *ytarget, c128 *dot_part = nullptr) {
        (void)o;
        const bool dot = dot_part != nullptr;
        auto &td = t_.td;
        const T *Sv = sval();
        const double sigma = cheb_theta_ / cheb_delta_;
        const int K = cheb_steps_;
        cpx<T> *buf[2];
        buf[K % 2] = ytarget;
        buf[(K + 1) % 2] = t_.w.get();
        double rho_prev = 1.0 / sigma;
        auto step = [&](int kk, const int *skip, int c0, int w, int dot_mode) {
            const double rho = 1.0 / (2.0 * sigma - rho_prev);
            const double c1 = rho * rho_prev, c2 = 2.0 * rho / cheb_delta_;
            const int mode = kk == 1 ? 0 : kk == 2 ? 1 : 2;
            launch_cheb_step<T>(st_, pr_, td, mode, c0, w, Sv, buf[kk % 2], t_.r.get(), buf[(kk + 1) % 2],
                                    skip, 1.0 / cheb_theta_, c1, c2, t_.part_d.get(), dot ? dot_part : nullptr,
                                    dot ? dot_mode : 0);
            rho_prev = rho;
        };
        // the K - 1 steps of each column block run back to back (columns are
        // independent); one event pair times them all
        const double vec = static_cast<double>(last_active_) * td.N * sizeof(cpx<T>);
        double bytes = 0.0;
        for (int k = 1; k < K; ++k) bytes += vec * (k == 1 ? 2 : k == 2 ? 3 : 4);
        const int cb = td.cb > 0 ? td.cb : td.Rp;
        int launches = 0;
        prof_.begin_group(st_, KP_CHEB);
        for (int c0 = 0; c0 < td.Rp; c0 += cb) {
            rho_prev = 1.0 / sigma;
            for (int k = 1; k < K; ++k, ++launches)
                step(k, t_.c_done.get(), c0, std::min(cb, td.Rp - c0), k == K - 1 ? 1 : 0);
        }
        prof_.end_group(st_, launches, bytes);
        k_cheb_check<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, t_.part_d.get(), inner_tol_ / cheb_rho_, 0, cs);
        // extra steps for the columns that failed the check (bytes counted
        // from the check's outcome are not known here: counted as zero)
        prof_.begin_group(st_, KP_CHEB);
        step(K, t_.c_inner_done.get(), 0, td.Rp, 0);
        step(K + 1, t_.c_inner_done.get(), 0, td.Rp, 2);
        prof_.end_group(st_, 2, 0.0);
        k_cheb_check<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, t_.part_d.get(), inner_tol_, 1, cs);
        GSC_HIP(hipGetLastError());
        inner_total_ += K - 1;
        return dot;
    }

    void inner_solve_cg(const gsc_opts &o, ColState cs, cpx<T> *y) {
        auto &td = t_.td;
        const dim3 eg(td.Rp / 64, td.G), eb(kBlock);
        int done_steps = 0;
        int chunk = inner_guess_;
        const T *Sv = sval();
        // algorithmic bytes per CG step over the columns still active
        const double vec = static_cast<double>(last_active_ > 0 ? last_active_ : td.R) * td.N * sizeof(cpx<T>);
        while (true) {
            for (int j = 0; j < chunk; ++j) {
                prof_.begin(st_, KP_SPMM_S, mat_bytes() + 2 * vec);
                launch_spmm_S<T>(st_, pr_, td, Sv, t_.d.get(), t_.w.get(), t_.c_inner_done.get(), t_.part_d.get());
                prof_.end(st_);
                k_cg_a<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.Gs, t_.part_d.get(), cs);
                prof_.begin(st_, KP_CG_UPDATE, 6 * vec);
                k_cg_update<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_inner_done.get(), t_.c_cg_first.get(),
                                                  t_.c_cg_a.get(), t_.d.get(), t_.w.get(), y, t_.res.get(),
                                                  t_.part_d.get());
                prof_.end(st_);
                k_cg_b<<<td.Rp, kBlock, 0, st_>>>(td.Rp, td.G, t_.part_d.get(), o.inner_max_iter, cs);
                prof_.begin(st_, KP_CG_DIR, 3 * vec);
                k_cg_dir<T><<<eg, eb, 0, st_>>>(td.N, td.Rp, td.Lr, t_.c_inner_done.get(), t_.c_cg_b.get(),
                                               t_.res.get(), t_.d.get());
                prof_.end(st_);
            }
            GSC_HIP(hipGetLastError());
            done_steps += chunk;
            const Status s = check_status(false);
            if (s.inner_pending == 0 || done_steps >= o.inner_max_iter) break;
            chunk = 2;
        }
        inner_total_ += done_steps;
        inner_guess_ = std::max(1, done_steps);
    }

    void flush(ColState cs, ShiftState ss, int n0, int n1, int only_sw, int nsw = -1) {
        auto &td = t_.td;
        if (prof_.on) flushes_.push_back({n0, n1, only_sw ? nsw : -1});
        constexpr int E = 1;
        dim3 grid(div_up(td.N, kBlock * E), td.Rp, 1);
        const size_t NR = static_cast<size_t>(td.N) * td.Rp;
        prof_.begin(st_, KP_SHIFT_UPDATE, 0.0);
#define GSC_FLUSH(MM)                                                                                        \
    k_flush<T, MM, E><<<grid, kBlock, 0, st_>>>(td.N, td.Rp, td.K, td.m, n0, n1, only_sw, cs, ss, \
                                                   t_.ringT.get(), NR, t_.X, ldk_x_, t_.P.get(), t_.ldk, td.R)
        if (td.m <= 1) GSC_FLUSH(1);
        else if (td.m <= 2) GSC_FLUSH(2);
        else if (td.m <= 4) GSC_FLUSH(4);
        else if (td.m <= 8) GSC_FLUSH(8);
        else GSC_FLUSH(16);
#undef GSC_FLUSH
        prof_.end(st_);
        GSC_HIP(hipGetLastError());
    }

    void proj_update(ColState cs, ShiftState ss, int slot, const cpx<T> *rp) {
        auto &td = t_.td;
        const int M = t_.Mu + t_.srow;
        const size_t shm = static_cast<size_t>(M) * sizeof(c128);
        prof_.begin(st_, KP_PROJ_UPDATE, 0.0);
        if (req_.vjp) {
            const int M = t_.Mu + t_.srow;
            k_proj_update_vjp<T><<<td.Rp, kBlock, shm, st_>>>(
                td.K, td.Rp, t_.Mu, t_.srow, slot, td.B, pr_.rowptr.get(), pr_.colidx.get(), pr_.S.get(), drhs_,
                t_.pidx.get(), cs, ss, rp, t_.h.get(), t_.dh.get(), req_.wE,
                req_.vjp_acc + static_cast<size_t>(r0_) * M * 3);
        } else {
            k_proj_update<T><<<td.Rp, kBlock, shm, st_>>>(td.K, td.Rp, t_.Mu, t_.srow, slot, td.B, pr_.rowptr.get(),
                                                         pr_.colidx.get(), pr_.S.get(), drhs_, t_.pidx.get(), cs, ss,
                                                         rp, t_.h.get(), t_.gacc.get());
        }
        prof_.end(st_);
        GSC_HIP(hipGetLastError());
    }

    Ctx &ctx_;
    Profiler &prof_ = ctx_.prof;
    DevBuf<unsigned long long> ctr_;
    const SolveRequest &req_;
    const Pair &pr_;
    const c128 *dz_;
    const int64_t *drhs_;
    const c128 *dB_;
    int r0_;
    bool full_;
    hipStream_t st_;
    Tile<T> t_;
    size_t ldk_x_ = 0;
    HostStatus hs_;
    int inner_guess_ = 8;
    int last_active_ = 0;
    int lz_steps_ = 0;
    double inner_tol_ = 1e-12;
    bool cheb_ok_ = false;
    double cheb_theta_ = 1.0, cheb_delta_ = 0.5, cheb_rho_ = 0.5, cheb_lo_ = 0.0, cheb_hi_ = 0.0;
    int cheb_steps_ = 0, cheb_max_ = 200;
    double inner_tol_base_ = 0.0;     // the fixed inner tolerance of the solve
    static constexpr double kRelaxCap = 1e-3;
    // mixed inner solve: precision flag, complex64 right-hand side (r after
    // each residual update, or the FP64 residual between rounds) and the two
    // alternating complex64 iterates; the plan of rounds
    bool mixed_ = false;
    bool r32_fresh_ = false;
    DevBuf<c64> mx_f_, mx_ya_, mx_yb_;
    std::vector<int> mx_plan_;
    static constexpr double kMxFloor = 1e-5;
    static constexpr double kMxReach = 4e-6;
    static constexpr double kMxSingle = 2e-6;
    static constexpr int kMxSafetySteps = 4;
    long long cheb_extra_ = 0;
    long long inner_total_ = 0;
    int switches_ = 0;
    long long shift_rhs_iters_ = 0;
    double worst_res_ = 0.0;
    int flags_ = 0;
};

template <> const double *TileSolver<double>::sval() const { return pr_.S.get(); }
template <> const double *TileSolver<double>::hval() const { return pr_.H.get(); }
template <> const float *TileSolver<float>::sval() const { return pr_.S32.get(); }
template <> const float *TileSolver<float>::hval() const { return pr_.H32.get(); }

// Inner S-solve tolerance: 1e-2 tol by default, floored by what the vector
// precision can reach (complex64 products cannot resolve residuals below a
// few ulps of FP32; asking for more stalls the outer iteration).
template <typename T> double default_inner_tol(const gsc_opts &o) {
    const double floor_t = std::is_same<T, float>::value ? 2e-6 : 1e-15;
    return o.inner_tol > 0 ? std::max(o.inner_tol, floor_t) : std::max(1e-2 * o.tol, floor_t);
}

int default_seed(const std::vector<double> &z, int K) {
    double lo = z[0], hi = z[0];
    for (int k = 0; k < K; ++k) { lo = std::min(lo, z[2 * k]); hi = std::max(hi, z[2 * k]); }
    const double mid = 0.5 * (lo + hi);
    int best = 0;
    for (int k = 1; k < K; ++k)
        if (std::fabs(z[2 * k] - mid) < std::fabs(z[2 * best] - mid)) best = k;
    return best;
}

template <typename T>
gsc_status solve_typed(Ctx &ctx, SolveRequest &req) {
    const Pair &pr = *req.pair;
    const gsc_opts &o = req.opts;
    hipStream_t st = ctx.stream;
    const int N = static_cast<int>(pr.n);
    const bool full = o.carry == GSC_CARRY_FULL;
    std::vector<double> zh(req.z, req.z + 2 * req.K);
    DevBuf<c128> dz(req.K);
    GSC_HIP(hipMemcpyAsync(dz.get(), zh.data(), zh.size() * sizeof(double), hipMemcpyHostToDevice, st));
    const int seed0 = o.seed_index >= 0 ? o.seed_index : default_seed(zh, req.K);
    double inner_tol = default_inner_tol<T>(o);

    // tile width: all rhs if memory allows
    int Rt = o.rhs_tile > 0 ? o.rhs_tile : req.R;
    // m = 16 unless asked otherwise: fewer passes over x^k, p^k for 2m
    // seed-sized ring vectors per column
    int m = o.fuse_steps > 0 ? std::min(o.fuse_steps, kMaxFuse) : (full ? kMaxFuse : 1);
    if (!full) m = 1;
    if (full && o.rhs_tile <= 0) {
        const size_t freeb = dev_usable_bytes();
        const double per_col = 2.0 * req.K * N * sizeof(cpx<T>) + (2.0 * m + 8.0) * N * sizeof(cpx<T>);
        const int fit = static_cast<int>(0.8 * static_cast<double>(freeb) / per_col);
        Rt = std::max(1, std::min(Rt, fit));
    }
    if (!full && o.rhs_tile <= 0) {
        const size_t freeb = dev_usable_bytes();
        const int M = (req.proj ? req.proj->M : 0) + 1;
        const double per_col = 10.0 * N * sizeof(cpx<T>) + static_cast<double>(req.K) * (M * 2.0 * 16 + 256.0);
        const int fit = static_cast<int>(0.6 * static_cast<double>(freeb) / per_col);
        Rt = std::max(64, std::min(Rt, fit));
    }
    Rt = std::max(1, std::min(Rt, req.R));
    // the shift-update pass launches one grid row per column of the tile
    // (at most 65535); wider requests run in several tiles
    if (full) Rt = std::min(Rt, 65472);

    std::vector<double> res_tmp;
    double *res_host = req.stats ? req.stats->res_recursive : nullptr;
    unsigned char *conv_host = req.stats ? req.stats->converged : nullptr;
    if (res_host == nullptr) {
        res_tmp.resize(static_cast<size_t>(req.K) * req.R);
        res_host = res_tmp.data();
    }
    hipEvent_t e0, e1;
    GSC_HIP(hipEventCreate(&e0));
    GSC_HIP(hipEventCreate(&e1));
    GSC_HIP(hipEventRecord(e0, st));
    int max_iters = 0, switches = 0;
    long long inner = 0, sri = 0;
    bool all_conv = true;
    for (int r0 = 0; r0 < req.R; r0 += Rt) {
        const int R = std::min(Rt, req.R - r0);
        const int Rp = (R + 63) / 64 * 64;
        DevBuf<int64_t> drhs;
        if (req.rhs_idx != nullptr) {
            std::vector<int64_t> h(Rp, 0);
            for (int c = 0; c < R; ++c) h[c] = req.rhs_idx[r0 + c];
            drhs.alloc(Rp);
            GSC_HIP(hipMemcpyAsync(drhs.get(), h.data(), Rp * sizeof(int64_t), hipMemcpyHostToDevice, st));
        }
        DevBuf<c128> dB;
        const c128 *Bptr = nullptr;
        if (req.rhs_idx == nullptr) {
            if (req.out_mem == GSC_MEM_DEVICE) {
                Bptr = reinterpret_cast<const c128 *>(req.B_dense) + static_cast<size_t>(r0) * N;
            } else {
                dB.alloc(static_cast<size_t>(R) * N);
                GSC_HIP(hipMemcpyAsync(dB.get(), req.B_dense + 2 * static_cast<size_t>(r0) * N,
                                       static_cast<size_t>(R) * N * sizeof(c128), hipMemcpyHostToDevice, st));
                Bptr = dB.get();
            }
        }
        TileSolver<T> ts(ctx, req, dz.get(), drhs.get(), Bptr, r0, R, Rp, m, full);
        ts.allocate();
        const int it = ts.run(o, inner_tol, seed0);
        ts.write_outputs(req.stats, res_host, conv_host, o.tol, req.R);
        if (full && req.stats && req.stats->res_true) ts.true_residual(req.stats->res_true, req.R);
        max_iters = std::max(max_iters, it);
        inner += ts.inner_total();
        switches += ts.switches();
        sri += ts.shift_rhs_iters();
        if (ts.worst_res() > o.tol || (ts.flags() & FLAG_INNER)) all_conv = false;
    }
    GSC_HIP(hipEventRecord(e1, st));
    GSC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GSC_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (req.stats) {
        req.stats->outer_iters = max_iters;
        req.stats->inner_iters = inner;
        req.stats->switches = switches;
        req.stats->restarts = full ? 0 : switches;
        req.stats->shift_rhs_iters = sri;
        req.stats->seconds = ms * 1e-3;
    }
    return all_conv ? GSC_OK : GSC_NOT_CONVERGED;
}

// ------------------------------------------------------------------ batched
struct BatchJob {
    SolveRequest *req = nullptr;
    int sys = 0, r0 = 0, R = 0;
    double work = 0.0;
};

template <typename T>
gsc_status batched_typed(Ctx &ctx, std::vector<SolveRequest> &reqs, int graph_iters, int max_streams,
                         std::vector<int> &iters_out) {
    // jobs: one per (system, rhs tile), longest first; tiles of at most 128
    // rhs by default (more, smaller jobs keep the streams evenly loaded:
    // batch32 2.5 % faster than whole systems as jobs, mixed and FP64)
    std::vector<BatchJob> jobs;
    for (size_t si = 0; si < reqs.size(); ++si) {
        SolveRequest &rq = reqs[si];
        const int Rt = rq.opts.rhs_tile > 0 ? rq.opts.rhs_tile : std::min(rq.R, kBatchTile);
        for (int r0 = 0; r0 < rq.R; r0 += Rt) {
            BatchJob j;
            j.req = &rq;
            j.sys = static_cast<int>(si);
            j.r0 = r0;
            j.R = std::min(Rt, rq.R - r0);
            j.work = static_cast<double>(rq.pair->n) * j.R * (rq.K + 64.0);
            jobs.push_back(j);
        }
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const BatchJob &a, const BatchJob &b) { return a.work > b.work; });
    const int ns = std::max(1, std::min<int>(max_streams, static_cast<int>(jobs.size())));
    // device memory the live jobs' workspaces may hold together
    const int mem_mb = reqs.front().opts.batch_mem_mb;
    double budget = mem_mb > 0 ? static_cast<double>(mem_mb) * 1048576.0
                               : 0.8 * static_cast<double>(dev_usable_bytes());
    std::vector<hipStream_t> streams(ns);
    for (auto &st : streams) GSC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct Live {
        std::unique_ptr<TileSolver<T>> ts;
        DevBuf<c128> dz;
        DevBuf<int64_t> drhs;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t ev = nullptr;
        DevBuf<Status> dstat;
        Status *hstat = nullptr;
        int n = 0, stream = -1;
        long long col_iters = 0;            // column-iterations accounted so far
        double bytes = 0.0, bytes_inner = 0.0, ws = 0.0;
        bool inflight = false, finished = false, graphed = false, held = false;
        gsc_opts o{};
    };
    std::vector<Live> live(jobs.size());
    auto capture = [graph_iters](Live &L, hipStream_t st) {
        const long long counted = L.ts->inner_total();   // capturing runs nothing
        GSC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int g = 0; g < graph_iters; ++g) L.ts->enqueue_projected_iteration(L.o, 0);
        GSC_HIP(hipStreamEndCapture(st, &L.graph));
        GSC_HIP(hipGraphInstantiate(&L.exec, L.graph, nullptr, nullptr, 0));
        L.ts->set_inner_total(counted);
    };
    // the handles of a job; its workspace (the tile solver's vectors) is
    // released separately
    auto drop_handles = [](Live &L) {
        if (L.exec) (void)hipGraphExecDestroy(L.exec);
        if (L.graph) (void)hipGraphDestroy(L.graph);
        if (L.ev) (void)hipEventDestroy(L.ev);
        if (L.hstat) (void)hipHostFree(L.hstat);
        L.exec = nullptr;
        L.graph = nullptr;
        L.ev = nullptr;
        L.hstat = nullptr;
    };
    auto release_workspace = [](Live &L) {
        L.ts.reset();
        L.dz.release();
        L.drhs.release();
        L.dstat.release();
        L.held = false;
    };
    // estimated device bytes of a job's workspace: the tile's vectors and
    // the per-(shift, column) scalars, coefficients and projections
    auto job_bytes = [](const BatchJob &jb) {
        const SolveRequest &rq = *jb.req;
        const double Rp = (jb.R + 63) / 64 * 64;
        const double NR = static_cast<double>(rq.pair->n) * Rp;
        const bool mx = std::is_same<T, double>::value && rq.opts.precision == GSC_MIXED;
        const double vec = (7.0 + (mx ? 1.5 : 0.0)) * NR * sizeof(cpx<T>);
        const int M = (rq.proj ? rq.proj->M : 0) + 1;
        const double KR = static_cast<double>(rq.K) * Rp;
        return vec + KR * (9.0 * 16.0 + 2.0 * M * 16.0) + 64.0 * Rp * 64.0;
    };
    const bool prof_was_on = ctx.prof.on;
    ctx.prof.on = false;   // no event nodes inside captured graphs
    gsc_status result = GSC_OK;
    iters_out.assign(reqs.size(), 0);
    std::vector<int> stream_busy(ns, 0);
    double live_bytes = 0.0;            // workspaces held (live and finished, not yet released)
    size_t next = 0, running = 0;
    try {
        // set-up of job j on stream si: workspace, first inner solve,
        // captured chunk of graph_iters iterations
        auto start = [&](size_t j, int si) {
            BatchJob &jb = jobs[j];
            SolveRequest &rq = *jb.req;
            Live &L = live[j];
            L.o = rq.opts;
            L.stream = si;
            hipStream_t st = streams[si];
            std::vector<double> zh(rq.z, rq.z + 2 * rq.K);
            L.dz.alloc(rq.K);
            GSC_HIP(hipMemcpyAsync(L.dz.get(), zh.data(), zh.size() * sizeof(double), hipMemcpyHostToDevice, st));
            const int Rp = (jb.R + 63) / 64 * 64;
            std::vector<int64_t> h(Rp, 0);
            for (int c = 0; c < jb.R; ++c) h[c] = rq.rhs_idx[jb.r0 + c];
            L.drhs.alloc(Rp);
            GSC_HIP(hipMemcpyAsync(L.drhs.get(), h.data(), Rp * sizeof(int64_t), hipMemcpyHostToDevice, st));
            const int seed0 = L.o.seed_index >= 0 ? L.o.seed_index : default_seed(zh, rq.K);
            const double inner_tol = default_inner_tol<T>(L.o);
            L.ts = std::make_unique<TileSolver<T>>(ctx, rq, L.dz.get(), L.drhs.get(), nullptr, jb.r0, jb.R, Rp, 1,
                                                   false);
            L.ts->set_stream(st);
            L.ts->allocate();
            L.held = true;
            L.ts->init_phase(L.o, inner_tol, seed0);
            GSC_HIP(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
            L.dstat.alloc(1);
            GSC_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.hstat), sizeof(Status), hipHostMallocDefault));
            if (L.ts->chebyshev_ready() && L.o.inner_method != 1) {
                // capture graph_iters outer iterations; replay until done
                capture(L, st);
                L.graphed = true;
            }
        };
        // outputs, statistics and handles of a finished job (its stream
        // is idle); the workspace stays until its room is needed
        auto finish = [&](size_t j) {
            Live &L = live[j];
            SolveRequest &rq = *jobs[j].req;
            double *res_host = rq.stats ? rq.stats->res_recursive : nullptr;
            unsigned char *conv_host = rq.stats ? rq.stats->converged : nullptr;
            L.ts->write_outputs(rq.stats, res_host, conv_host, L.o.tol, rq.R);
            iters_out[jobs[j].sys] = std::max(iters_out[jobs[j].sys], std::min(L.n, L.o.max_iter));
            if (rq.stats) {
                rq.stats->outer_iters = iters_out[jobs[j].sys];
                rq.stats->inner_iters += L.ts->inner_total();
                rq.stats->shift_rhs_iters += L.ts->shift_rhs_iters();
                rq.stats->alg_bytes += L.bytes;
                rq.stats->alg_bytes_inner += L.bytes_inner;
            }
            if (L.ts->worst_res() > L.o.tol || (L.ts->flags() & FLAG_INNER)) result = GSC_NOT_CONVERGED;
            drop_handles(L);
            L.finished = true;
            stream_busy[L.stream] = 0;
        };
        while (next < jobs.size() || running > 0) {
            bool progress = false;
            // start the next jobs while a stream is free and their
            // workspaces fit beside the ones held; finished jobs give back
            // their room first (a job always starts when none is live)
            while (next < jobs.size()) {
                int si = -1;
                for (int k = 0; k < ns; ++k)
                    if (!stream_busy[k]) { si = k; break; }
                if (si < 0) break;
                const double need = job_bytes(jobs[next]);
                if (live_bytes + need > budget) {
                    for (size_t j = 0; j < next && live_bytes + need > budget; ++j)
                        if (live[j].finished && live[j].held) {
                            release_workspace(live[j]);
                            live_bytes -= live[j].ws;
                        }
                }
                if (running > 0 && live_bytes + need > budget) break;
                live[next].ws = need;
                live_bytes += need;
                stream_busy[si] = 1;
                ++running;
                try {
                    start(next, si);
                } catch (const Error &e) {
                    // the device is fuller than the estimate: with other
                    // jobs live, undo this start and wait for their room
                    if (e.code != GSC_E_NOMEM || running == 1) throw;
                    (void)hipGetLastError();
                    (void)hipStreamSynchronize(streams[si]);
                    drop_handles(live[next]);
                    release_workspace(live[next]);
                    live_bytes -= need;
                    budget = live_bytes;
                    stream_busy[si] = 0;
                    --running;
                    break;
                }
                ++next;
                progress = true;
            }
            // keep one chunk in flight per live job, poll completion events
            for (size_t j = 0; j < next; ++j) {
                Live &L = live[j];
                if (L.finished) continue;
                hipStream_t st = streams[L.stream];
                if (!L.inflight) {
                    if (L.graphed) {
                        GSC_HIP(hipGraphLaunch(L.exec, st));
                        L.n += graph_iters;
                        L.ts->set_inner_total(L.ts->inner_total() +
                                              static_cast<long long>(graph_iters) * L.ts->cheb_steps_per_solve());
                    } else {
                        L.ts->enqueue_projected_iteration(L.o, L.n);
                        L.n += 1;
                    }
                    L.ts->enqueue_status(L.dstat.get(), L.hstat);
                    GSC_HIP(hipEventRecord(L.ev, st));
                    L.inflight = true;
                    progress = true;
                    continue;
                }
                const hipError_t q = hipEventQuery(L.ev);
                if (q == hipErrorNotReady) continue;
                GSC_HIP(q);
                L.inflight = false;
                progress = true;
                const Status s = *L.hstat;
                L.ts->note_status(s);
                // algorithmic bytes of the iterations since the last poll,
                // with the inner plan they ran with
                const double dci = static_cast<double>(s.col_iters - L.col_iters);
                L.col_iters = s.col_iters;
                L.bytes += dci * L.ts->col_iter_bytes();
                L.bytes_inner += dci * L.ts->col_iter_inner_bytes();
                if (s.active_cols == 0 || L.n >= L.o.max_iter) {
                    finish(j);
                    --running;
                } else if (L.o.inner_relax && L.ts->relax_from_status(s, L.graphed) && L.graphed) {
                    // the graph holds the Chebyshev step count: capture anew
                    (void)hipGraphExecDestroy(L.exec);
                    (void)hipGraphDestroy(L.graph);
                    L.exec = nullptr;
                    L.graph = nullptr;
                    capture(L, st);
                }
            }
            if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        for (auto &st : streams) GSC_HIP(hipStreamSynchronize(st));
    } catch (...) {
        ctx.prof.on = prof_was_on;
        // other jobs' graphs and their status copies may still be in
        // flight: drain every stream before anything they use is released
        for (auto &st : streams) (void)hipStreamSynchronize(st);
        for (auto &L : live) drop_handles(L);
        for (auto &st : streams) (void)hipStreamDestroy(st);
        throw;
    }
    ctx.prof.on = prof_was_on;
    for (auto &L : live) drop_handles(L);
    for (auto &st : streams) (void)hipStreamDestroy(st);
    return result;
}

// Generalised Lanczos for the unit right-hand sides of one request, in tiles
// of processes (two per column).
template <typename T>
gsc_status lanczos_typed(Ctx &ctx, LanczosRequest &req) {
    const Pair &pr = *req.pair;
    const gsc_opts &o = req.opts;
    hipStream_t st = ctx.stream;
    const int N = static_cast<int>(pr.n);
    std::vector<double> zh(req.z, req.z + 2 * req.K);
    DevBuf<c128> dz(req.K);
    GSC_HIP(hipMemcpyAsync(dz.get(), zh.data(), zh.size() * sizeof(double), hipMemcpyHostToDevice, st));
    const double inner_tol = default_inner_tol<T>(o);
    int Pt = o.rhs_tile > 0 ? o.rhs_tile : req.P;
    if (o.rhs_tile <= 0) {
        const size_t freeb = dev_usable_bytes();
        // per column: ~12 vectors plus coefficient rows of two processes
        const double per_col = 12.0 * N * sizeof(cpx<T>) + 4.0 * req.m_max * sizeof(double) + 32.0 * req.K;
        const int fit = static_cast<int>(0.6 * static_cast<double>(freeb) / per_col);
        Pt = std::max(128, std::min(Pt, 2 * fit));
    }
    Pt = std::max(2, std::min(Pt, req.P));
    Pt += Pt & 1;
    // device output [K][P]
    DevBuf<c128> gown;
    c128 *gout = nullptr;
    if (req.out_mem == GSC_MEM_DEVICE) {
        gout = reinterpret_cast<c128 *>(req.G_diag);
    } else {
        gown.alloc(static_cast<size_t>(req.K) * req.P);
        gout = gown.get();
    }
    hipEvent_t e0, e1;
    GSC_HIP(hipEventCreate(&e0));
    GSC_HIP(hipEventCreate(&e1));
    GSC_HIP(hipEventRecord(e0, st));
    int max_steps = 0;
    long long inner = 0, sri = 0;
    for (int p0 = 0; p0 < req.P; p0 += Pt) {
        const int P = std::min(Pt, req.P - p0);
        const int ncol = (P + 1) / 2;
        const int Rp = (ncol + 63) / 64 * 64;
        std::vector<int64_t> hr(2 * static_cast<size_t>(Rp), -1);
        for (int p = 0; p < P; ++p) hr[p] = req.rhs_idx[p0 + p];
        DevBuf<int64_t> drhs(hr.size());
        GSC_HIP(hipMemcpyAsync(drhs.get(), hr.data(), hr.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        SolveRequest sreq;
        sreq.pair = req.pair;
        sreq.K = req.K;
        sreq.z = req.z;
        sreq.R = ncol;
        sreq.opts = o;
        sreq.opts.carry = GSC_CARRY_PROJECTED;
        sreq.out_mem = req.out_mem;
        TileSolver<T> ts(ctx, sreq, dz.get(), nullptr, nullptr, 0, ncol, Rp, 1, false);
        ts.allocate();
        const size_t PR = 2 * static_cast<size_t>(Rp);
        DevBuf<double> a(PR * req.m_max), b(PR * req.m_max), vj(PR);
        DevBuf<int> steps(PR);
        ts.run_lanczos(o, inner_tol, drhs.get(), P, req.m_max, req.tol, req.check_every, a.get(), b.get(),
                       steps.get(), vj.get(), gout, req.P, p0);
        std::vector<int> hs(PR);
        GSC_HIP(hipMemcpyAsync(hs.data(), steps.get(), PR * sizeof(int), hipMemcpyDeviceToHost, st));
        if (req.coef_a) {
            GSC_HIP(hipMemcpyAsync(req.coef_a + static_cast<size_t>(p0) * req.m_max, a.get(),
                                   static_cast<size_t>(P) * req.m_max * sizeof(double), hipMemcpyDeviceToHost, st));
        }
        if (req.coef_b) {
            GSC_HIP(hipMemcpyAsync(req.coef_b + static_cast<size_t>(p0) * req.m_max, b.get(),
                                   static_cast<size_t>(P) * req.m_max * sizeof(double), hipMemcpyDeviceToHost, st));
        }
        GSC_HIP(hipStreamSynchronize(st));
        for (int p = 0; p < P; ++p) {
            if (req.steps) req.steps[p0 + p] = hs[p];
            max_steps = std::max(max_steps, hs[p]);
            sri += static_cast<long long>(hs[p]) * req.K;
        }
        inner += ts.inner_total();
    }
    if (req.out_mem != GSC_MEM_DEVICE) {
        GSC_HIP(hipMemcpyAsync(req.G_diag, gout, static_cast<size_t>(req.K) * req.P * sizeof(c128),
                               hipMemcpyDeviceToHost, st));
    }
    GSC_HIP(hipEventRecord(e1, st));
    GSC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GSC_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (req.stats) {
        req.stats->outer_iters = max_steps;
        req.stats->inner_iters = inner;
        req.stats->switches = 0;
        req.stats->restarts = 0;
        req.stats->shift_rhs_iters = sri;
        req.stats->seconds = ms * 1e-3;
    }
    return max_steps >= req.m_max && req.check_every > 0 ? GSC_NOT_CONVERGED : GSC_OK;
}

}  // namespace

// GSC_C64 runs the whole seed process in complex64 (TileSolver<float>);
// GSC_MIXED keeps it in FP64 and runs the inner S-solve in complex64 rounds
// refined in FP64 (TileSolver<double>); both read the FP32 copy of S.
gsc_status run_batched(Ctx &ctx, std::vector<SolveRequest> &reqs, int graph_iters, int max_streams,
                       std::vector<int> &iters) {
    bool c64 = false;
    for (auto &r : reqs) {
        c64 |= r.opts.precision == GSC_C64;
        if (r.opts.precision != GSC_FP64) ensure_f32(const_cast<Pair &>(*r.pair));
    }
    if (c64) return batched_typed<float>(ctx, reqs, graph_iters, max_streams, iters);
    return batched_typed<double>(ctx, reqs, graph_iters, max_streams, iters);
}

gsc_status run_solve(Ctx &ctx, SolveRequest &req) {
    if (req.opts.precision != GSC_FP64) ensure_f32(const_cast<Pair &>(*req.pair));
    if (req.opts.precision == GSC_C64) return solve_typed<float>(ctx, req);
    return solve_typed<double>(ctx, req);
}

gsc_status run_lanczos(Ctx &ctx, LanczosRequest &req) {
    if (req.opts.precision != GSC_FP64) ensure_f32(const_cast<Pair &>(*req.pair));
    if (req.opts.precision == GSC_C64) return lanczos_typed<float>(ctx, req);
    return lanczos_typed<double>(ctx, req);
}

}  // namespace gsc
