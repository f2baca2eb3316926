// Block-sparse products with H and S for many right-hand sides at once.
//
// One wave owns 64 consecutive columns and walks one block row at a time;
// the B x B blocks of S and H are wave-uniform (scalar loads), the gathered
// x rows are 64 contiguous complex values per orbital (one coalesced
// 1 KiB (FP64) transaction per orbital row).  No MFMA: per stored value the
// product does 2 (S only) or 4 (S and H) FMAs per complex column against
// >= 16 bytes of vector traffic, far below the FP64 ridge.
#include <algorithm>

#include "spmm.h"

namespace gsc {

// q = zs_c * (S p) - H p for every active column c, plus the per-column
// unconjugated partial dot  sum_i p_i q_i  (the denominator of alpha,
// eq. CGp:r with the S-bilinear form) of this row group.
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_spmm_seed(
    int nb, int Rp, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const T *__restrict__ Hv, const cpx<T> *__restrict__ p,
    cpx<T> *__restrict__ q, const c128 *__restrict__ z, const int *__restrict__ seed,
    const int *__restrict__ skip, c128 *__restrict__ partial) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int col = cx * 64 + lane;
    const bool act = skip == nullptr || !skip[col];
    c128 zs = act ? z[seed[col]] : c128{0, 0};
    const cpx<T> zt = ccast<T>(zs);
    c128 dot{0.0, 0.0};
    // rows of this wave: every row group takes one row per wave per step, so
    // the groups advance together (step i covers rows [i*4*Gs, (i+1)*4*Gs))
    // and the rows in flight on an XCD stay within one window, however many
    // rows a group holds
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + w; I < nb; I += row_step) {
            cpx<T> aS[B], aH[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = {0, 0}; aH[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            // loads of finished columns are masked off (their lines are not
            // fetched); their registers keep stale values that are never used
            cpx<T> x[B];
#pragma unroll
            for (int c = 0; c < B; ++c) x[c] = {0, 0};
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                const T *hb = Hv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c) x[c] = p[static_cast<size_t>(J * B + c) * Rp + col];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const T s = sb[a * B + c], h = hb[a * B + c];
                        aS[a].re = fma(s, x[c].re, aS[a].re);
                        aS[a].im = fma(s, x[c].im, aS[a].im);
                        aH[a].re = fma(h, x[c].re, aH[a].re);
                        aH[a].im = fma(h, x[c].im, aH[a].im);
                    }
                }
            }
            // the row's own p values (diagonal block) are re-read: an L2 hit,
            // cheaper than holding them in registers through the row
#pragma unroll
            for (int a = 0; a < B; ++a) {
                const cpx<T> v = zt * aS[a] - aH[a];
                if (act) {
                    const size_t e = static_cast<size_t>(I * B + a) * Rp + col;
                    q[e] = v;
                    dot = dot + ccast<double>(p[e]) * ccast<double>(v);
                }
            }
        }
    }
    __shared__ c128 red[kWavesPerBlock][64];
    red[w][lane] = dot;
    __syncthreads();
    if (threadIdx.x < 64) {
        c128 s = red[0][lane];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) s = s + red[k][lane];
        partial[static_cast<size_t>(g) * Rp + col] = s;
    }
}

// w = S d for the columns whose inner solve is still running, plus the
// per-column partial  Re(d^H S d)  (the CG curvature; S real symmetric).
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_spmm_S(
    int nb, int Rp, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const cpx<T> *__restrict__ d, cpx<T> *__restrict__ wout,
    const int *__restrict__ skip, double *__restrict__ partial) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = cx * 64 + lane;
    const bool act = !skip[col];
    double dot = 0.0;
    // rows of this wave: every row group takes one row per wave per step, so
    // the groups advance together (step i covers rows [i*4*Gs, (i+1)*4*Gs))
    // and the rows in flight on an XCD stay within one window, however many
    // rows a group holds
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            cpx<T> aS[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = {0, 0}; own[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            // loads of finished columns are masked off (their lines are not
            // fetched); their registers keep stale values that are never used
            cpx<T> x[B];
#pragma unroll
            for (int c = 0; c < B; ++c) x[c] = {0, 0};
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c) x[c] = d[static_cast<size_t>(J * B + c) * Rp + col];
                }
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) own[c] = x[c];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const T s = sb[a * B + c];
                        aS[a].re = fma(s, x[c].re, aS[a].re);
                        aS[a].im = fma(s, x[c].im, aS[a].im);
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < B; ++a) {
                if (act) {
                    wout[static_cast<size_t>(I * B + a) * Rp + col] = aS[a];
                    dot += static_cast<double>(own[a].re) * aS[a].re +
                           static_cast<double>(own[a].im) * aS[a].im;
                }
            }
        }
    }
    __shared__ double red[kWavesPerBlock][64];
    red[wv][lane] = dot;
    __syncthreads();
    if (threadIdx.x < 64) {
        double s = red[0][lane];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) s += red[k][lane];
        partial[static_cast<size_t>(g) * Rp + col] = s;
    }
}

// ------------------------------------------------------------------ Chebyshev step
// One step of the Chebyshev iteration for S y = r on the interval
// [theta - delta, theta + delta] fused with the product, in the three-term
// form (see cheb_update): one gathered vector (y_k, or r in the first
// step), r and y_{k-1} streamed, y_{k+1} written over y_{k-1}, and a
// partial ||r - S y_k||^2.  A launch covers the columns [col0, col0 +
// 64 gridDim.x) of the Rp-wide tile.  DOT: the step is a column's last, and
// the partial of y_{k+1}^T r (unconjugated: the next rho of the outer
// iteration, eq. CGp:p) goes to dpart as well, for every column
// (dot_active_only = 0) or only for the columns that take this step.
template <typename T, int B, int MODE, bool NT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_cheb_step(
    int nb, int Rp, int col0, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const cpx<T> *__restrict__ y, const cpx<T> *__restrict__ r,
    cpx<T> *__restrict__ yio, const int *__restrict__ skip, T inv_theta, T c1, T c2,
    double *__restrict__ partial, c128 *__restrict__ dpart, int dot_active_only) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = col0 + cx * 64 + lane;
    const bool act = !skip[col];
    double acc2 = 0.0;
    c128 dacc{0.0, 0.0};
    // rows of this wave: every row group takes one row per wave per step, so
    // the groups advance together (step i covers rows [i*4*Gs, (i+1)*4*Gs))
    // and the rows in flight on an XCD stay within one window, however many
    // rows a group holds
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    const cpx<T> *x = MODE == 0 ? r : y;
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            cpx<T> aS[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = {0, 0}; own[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            // loads of finished columns are masked off (their lines are not
            // fetched); their registers keep stale values that are never used
            cpx<T> xv[B];
#pragma unroll
            for (int c = 0; c < B; ++c) xv[c] = {0, 0};
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c) xv[c] = x[static_cast<size_t>(J * B + c) * Rp + col];
                }
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) own[c] = xv[c];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const T sv = sb[a * B + c];
                        aS[a].re = fma(sv, xv[c].re, aS[a].re);
                        aS[a].im = fma(sv, xv[c].im, aS[a].im);
                    }
                }
            }
            if (!act) continue;
#pragma unroll
            for (int a = 0; a < B; ++a)
                acc2 += cheb_update<T, MODE, NT>(own[a], aS[a], r, yio, static_cast<size_t>(I * B + a) * Rp + col,
                                                 inv_theta, c1, c2, DOT ? &dacc : nullptr);
        }
    }
    __shared__ double red[kWavesPerBlock][64];
    red[wv][lane] = acc2;
    if constexpr (DOT) {
        __shared__ c128 redc[kWavesPerBlock][64];
        redc[wv][lane] = dacc;
        __syncthreads();
        if (threadIdx.x < 64 && (act || !dot_active_only)) {
            c128 t = redc[0][lane];
#pragma unroll
            for (int k = 1; k < kWavesPerBlock; ++k) t = t + redc[k][lane];
            dpart[static_cast<size_t>(g) * Rp + col] = t;
        }
    } else {
        __syncthreads();
    }
    if (threadIdx.x < 64) {
        double t = red[0][lane];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) t += red[k][lane];
        partial[static_cast<size_t>(g) * Rp + col] = t;
    }
}

template <typename T>
void launch_cheb_step(hipStream_t st, const Pair &pr, const TileDims &td, int mode, int col0, int ncols,
                      const T *Sv, const cpx<T> *y, const cpx<T> *r, cpx<T> *yio, const int *skip,
                      double inv_theta, double c1, double c2, double *partial, c128 *dpart, int dot_mode) {
    GSC_REQUIRE(col0 % 64 == 0 && ncols % 64 == 0 && ncols > 0 && col0 + ncols <= td.Rp,
                "Chebyshev column block outside the tile");
    GSC_REQUIRE(dot_mode == 0 || dpart != nullptr, "the fused dot needs its partials");
    dim3 grid(ncols / 64, td.Gs), block(kBlock);
    const T it = static_cast<T>(inv_theta), a = static_cast<T>(c1), b = static_cast<T>(c2);
#define GSC_CHEB_D(BB, M, N, D)                                                                                   \
    k_cheb_step<T, BB, M, N, D><<<grid, block, 0, st>>>(td.nb, td.Rp, col0, pr.rowptr.get(), pr.colidx.get(), Sv, \
                                                        y, r, yio, skip, it, a, b, partial, dpart, dot_mode == 2)
#define GSC_CHEB(BB, M, N) \
    if (dot_mode) GSC_CHEB_D(BB, M, N, true); else GSC_CHEB_D(BB, M, N, false);
#define GSC_CHEB_N(BB, M) \
    if (td.nt) { GSC_CHEB(BB, M, true) } else { GSC_CHEB(BB, M, false) }
#define GSC_CHEB_B(BB) \
    if (mode == 0) { GSC_CHEB_N(BB, 0) } else if (mode == 1) { GSC_CHEB_N(BB, 1) } else { GSC_CHEB_N(BB, 2) }
    if (pr.B == 4) { GSC_CHEB_B(4) } else { GSC_CHEB_B(6) }
#undef GSC_CHEB_B
#undef GSC_CHEB_N
#undef GSC_CHEB
#undef GSC_CHEB_D
    GSC_HIP(hipGetLastError());
}

template void launch_cheb_step<double>(hipStream_t, const Pair &, const TileDims &, int, int, int, const double *,
                                       const c128 *, const c128 *, c128 *, const int *, double, double, double,
                                       double *, c128 *, int);
template void launch_cheb_step<float>(hipStream_t, const Pair &, const TileDims &, int, int, int, const float *,
                                      const c64 *, const c64 *, c64 *, const int *, double, double, double,
                                      double *, c128 *, int);

// ------------------------------------------------------------------ mixed inner solve
// Complex64 rounds of the inner solve S Y = r refined in FP64 (iterative
// refinement).  Inside a round the iterates y live in complex64 and each step
// runs in FP32 arithmetic against the FP32 copy of S, solving S y = f for the
// round's right-hand side f (complex64).  The round's last step (FIN) does not
// store its iterate: it adds it to the FP64 solution Y (FIN 1: Y = y, FIN 2:
// Y += y), and with DOT it also forms the partial of Y^T r (unconjugated,
// FP64: the next rho of the outer iteration, eq. CGp:p) from the FP64 r.
// Between rounds k_mx_resid forms the next right-hand side f = r - S Y in
// FP64, so rounding in the complex64 rounds limits only how fast the
// refinement converges, not where it ends.
template <int B, int MODE, int FIN, bool DOT>
__global__ __launch_bounds__(kBlock) void k_cheb_mx(
    int nb, int Rp, int col0, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const float *__restrict__ Sv, const c64 *__restrict__ y, const c64 *__restrict__ f, c64 *__restrict__ yio,
    c128 *__restrict__ Y, const c128 *__restrict__ r, const int *__restrict__ skip, float inv_theta, float c1,
    float c2, double *__restrict__ partial, c128 *__restrict__ dpart, int dot_active_only) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = col0 + cx * 64 + lane;
    const bool act = !skip[col];
    double acc2 = 0.0;
    c128 dacc{0.0, 0.0};
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    const c64 *x = MODE == 0 ? f : y;
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            c64 aS[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = {0, 0}; own[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            c64 xv[B];
#pragma unroll
            for (int c = 0; c < B; ++c) xv[c] = {0, 0};
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const float *sb = Sv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c) xv[c] = x[static_cast<size_t>(J * B + c) * Rp + col];
                }
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) own[c] = xv[c];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const float sv = sb[a * B + c];
                        aS[a].re = fmaf(sv, xv[c].re, aS[a].re);
                        aS[a].im = fmaf(sv, xv[c].im, aS[a].im);
                    }
                }
            }
            if (!act) continue;
#pragma unroll
            for (int a = 0; a < B; ++a) {
                const size_t e = static_cast<size_t>(I * B + a) * Rp + col;
                double res2;
                c64 rv;
                const c64 ynew = cheb_next<float, MODE, false>(own[a], aS[a], f, yio, e, inv_theta, c1, c2, res2, rv);
                acc2 += res2;
                if constexpr (FIN == 0) {
                    yio[e] = ynew;
                } else {
                    c128 v = ccast<double>(ynew);
                    if constexpr (FIN == 2) v = Y[e] + v;
                    Y[e] = v;
                    if constexpr (DOT) dacc = dacc + v * r[e];
                }
            }
        }
    }
    __shared__ double red[kWavesPerBlock][64];
    red[wv][lane] = acc2;
    if constexpr (DOT) {
        __shared__ c128 redc[kWavesPerBlock][64];
        redc[wv][lane] = dacc;
        __syncthreads();
        if (threadIdx.x < 64 && (act || !dot_active_only)) {
            c128 t = redc[0][lane];
#pragma unroll
            for (int k = 1; k < kWavesPerBlock; ++k) t = t + redc[k][lane];
            dpart[static_cast<size_t>(g) * Rp + col] = t;
        }
    } else {
        __syncthreads();
    }
    if (threadIdx.x < 64) {
        double t = red[0][lane];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) t += red[k][lane];
        partial[static_cast<size_t>(g) * Rp + col] = t;
    }
}

// k_cheb_mx with two columns per lane: a wave covers 128 columns and every
// gathered load moves 16 bytes per lane (two complex64), half the load
// instructions per byte of the one-column form.  Same arithmetic per
// column, same order.
template <int B, int MODE, int FIN, bool DOT>
__global__ __launch_bounds__(kBlock) void k_cheb_mx2(
    int nb, int Rp, int col0, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const float *__restrict__ Sv, const c64 *__restrict__ y, const c64 *__restrict__ f, c64 *__restrict__ yio,
    c128 *__restrict__ Y, const c128 *__restrict__ r, const int *__restrict__ skip, float inv_theta, float c1,
    float c2, double *__restrict__ partial, c128 *__restrict__ dpart, int dot_active_only) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = col0 + cx * 128 + 2 * lane;
    const bool act0 = !skip[col], act1 = !skip[col + 1];
    const bool act = act0 || act1;
    double acc20 = 0.0, acc21 = 0.0;
    c128 dacc0{0.0, 0.0}, dacc1{0.0, 0.0};
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    const c64 *x = MODE == 0 ? f : y;
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            c64 a0[B], a1[B], o0[B], o1[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { a0[a] = {0, 0}; a1[a] = {0, 0}; o0[a] = {0, 0}; o1[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            float4 xv[B];
#pragma unroll
            for (int c = 0; c < B; ++c) xv[c] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const float *sb = Sv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c)
                        xv[c] = *reinterpret_cast<const float4 *>(x + static_cast<size_t>(J * B + c) * Rp + col);
                }
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) { o0[c] = {xv[c].x, xv[c].y}; o1[c] = {xv[c].z, xv[c].w}; }
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const float sv = sb[a * B + c];
                        a0[a].re = fmaf(sv, xv[c].x, a0[a].re);
                        a0[a].im = fmaf(sv, xv[c].y, a0[a].im);
                        a1[a].re = fmaf(sv, xv[c].z, a1[a].re);
                        a1[a].im = fmaf(sv, xv[c].w, a1[a].im);
                    }
                }
            }
            if (!act) continue;
#pragma unroll
            for (int a = 0; a < B; ++a) {
                const size_t e = static_cast<size_t>(I * B + a) * Rp + col;
                double r20, r21;
                c64 rv0, rv1;
                const c64 n0 = cheb_next<float, MODE, false>(o0[a], a0[a], f, yio, e, inv_theta, c1, c2, r20, rv0);
                const c64 n1 = cheb_next<float, MODE, false>(o1[a], a1[a], f, yio, e + 1, inv_theta, c1, c2, r21, rv1);
                if (act0) acc20 += r20;
                if (act1) acc21 += r21;
                if constexpr (FIN == 0) {
                    if (act0 && act1) {
                        *reinterpret_cast<float4 *>(yio + e) = make_float4(n0.re, n0.im, n1.re, n1.im);
                    } else {
                        if (act0) yio[e] = n0;
                        if (act1) yio[e + 1] = n1;
                    }
                } else {
                    if (act0) {
                        c128 v = ccast<double>(n0);
                        if constexpr (FIN == 2) v = Y[e] + v;
                        Y[e] = v;
                        if constexpr (DOT) dacc0 = dacc0 + v * r[e];
                    }
                    if (act1) {
                        c128 v = ccast<double>(n1);
                        if constexpr (FIN == 2) v = Y[e + 1] + v;
                        Y[e + 1] = v;
                        if constexpr (DOT) dacc1 = dacc1 + v * r[e + 1];
                    }
                }
            }
        }
    }
    __shared__ double red[2][kWavesPerBlock][64];
    red[0][wv][lane] = acc20;
    red[1][wv][lane] = acc21;
    if constexpr (DOT) {
        __shared__ c128 redc[2][kWavesPerBlock][64];
        redc[0][wv][lane] = dacc0;
        redc[1][wv][lane] = dacc1;
        __syncthreads();
        if (threadIdx.x < 128) {
            const int h = threadIdx.x >> 6, ln = threadIdx.x & 63;
            const int cc = col0 + cx * 128 + 2 * ln + h;
            if (!skip[cc] || !dot_active_only) {
                c128 t = redc[h][0][ln];
#pragma unroll
                for (int k = 1; k < kWavesPerBlock; ++k) t = t + redc[h][k][ln];
                dpart[static_cast<size_t>(g) * Rp + cc] = t;
            }
        }
    } else {
        __syncthreads();
    }
    if (threadIdx.x < 128) {
        const int h = threadIdx.x >> 6, ln = threadIdx.x & 63;
        const int cc = col0 + cx * 128 + 2 * ln + h;
        double t = red[h][0][ln];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) t += red[h][k][ln];
        partial[static_cast<size_t>(g) * Rp + cc] = t;
    }
}

// f = r - S Y in FP64 (S, Y, r in FP64), stored in complex64 as the
// right-hand side of the next complex64 round; partial ||f||^2.
template <int B>
__global__ __launch_bounds__(kBlock) void k_mx_resid(
    int nb, int Rp, int col0, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const double *__restrict__ Sv, const c128 *__restrict__ Y, const c128 *__restrict__ r, c64 *__restrict__ f,
    const int *__restrict__ skip, double *__restrict__ partial) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = col0 + cx * 64 + lane;
    const bool act = !skip[col];
    double acc2 = 0.0;
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            c128 aS[B];
#pragma unroll
            for (int a = 0; a < B; ++a) aS[a] = {0, 0};
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            c128 xv[B];
#pragma unroll
            for (int c = 0; c < B; ++c) xv[c] = {0, 0};
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const double *sb = Sv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c) xv[c] = Y[static_cast<size_t>(J * B + c) * Rp + col];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const double sv = sb[a * B + c];
                        aS[a].re = fma(sv, xv[c].re, aS[a].re);
                        aS[a].im = fma(sv, xv[c].im, aS[a].im);
                    }
                }
            }
            if (!act) continue;
#pragma unroll
            for (int a = 0; a < B; ++a) {
                const size_t e = static_cast<size_t>(I * B + a) * Rp + col;
                const c128 d = r[e] - aS[a];
                f[e] = ccast<float>(d);
                acc2 += d.re * d.re + d.im * d.im;
            }
        }
    }
    __shared__ double red[kWavesPerBlock][64];
    red[wv][lane] = acc2;
    __syncthreads();
    if (threadIdx.x < 64) {
        double t = red[0][lane];
#pragma unroll
        for (int k = 1; k < kWavesPerBlock; ++k) t += red[k][lane];
        partial[static_cast<size_t>(g) * Rp + col] = t;
    }
}

void launch_cheb_mx(hipStream_t st, const Pair &pr, const TileDims &td, int mode, int fin, bool dot, int col0,
                    int ncols, const float *Sv, const c64 *y, const c64 *f, c64 *yio, c128 *Y, const c128 *r,
                    const int *skip, double inv_theta, double c1, double c2, double *partial, c128 *dpart,
                    int dot_active_only) {
    GSC_REQUIRE(col0 % 64 == 0 && ncols % 64 == 0 && ncols > 0 && col0 + ncols <= td.Rp,
                "Chebyshev column block outside the tile");
    GSC_REQUIRE(mode >= 0 && mode <= 2 && fin >= 0 && fin <= 2, "bad mixed Chebyshev step");
    GSC_REQUIRE(!dot || (fin > 0 && dpart != nullptr && r != nullptr), "the fused dot needs a final step");
    GSC_REQUIRE(fin == 0 || Y != nullptr, "a final step needs the FP64 solution");
    const float it = static_cast<float>(inv_theta), a = static_cast<float>(c1), b = static_cast<float>(c2);
    // 128-column pieces with two columns per lane, a 64-column tail with one
    const int n2 = ncols / 128 * 128;
    const dim3 block(kBlock);
    if (n2 > 0) {
        const dim3 grid(n2 / 128, td.Gs);
#define GSC_MX(BB, M, F, D)                                                                                    \
        k_cheb_mx2<BB, M, F, D><<<grid, block, 0, st>>>(td.nb, td.Rp, col0, pr.rowptr.get(), pr.colidx.get(), \
                                                        Sv, y, f, yio, Y, r, skip, it, a, b, partial, dpart,  \
                                                        dot_active_only)
#define GSC_MX_F(BB, M)                                                              \
    if (fin == 0) { GSC_MX(BB, M, 0, false); }                                       \
    else if (fin == 1) { if (dot) GSC_MX(BB, M, 1, true); else GSC_MX(BB, M, 1, false); } \
    else { if (dot) GSC_MX(BB, M, 2, true); else GSC_MX(BB, M, 2, false); }
#define GSC_MX_B(BB) \
    if (mode == 0) { GSC_MX_F(BB, 0) } else if (mode == 1) { GSC_MX_F(BB, 1) } else { GSC_MX_F(BB, 2) }
        if (pr.B == 4) { GSC_MX_B(4) } else { GSC_MX_B(6) }
#undef GSC_MX_B
#undef GSC_MX_F
#undef GSC_MX
    }
    if (n2 == ncols) {
        GSC_HIP(hipGetLastError());
        return;
    }
    const int c0 = col0 + n2;
    const dim3 grid((ncols - n2) / 64, td.Gs);
#define GSC_MX(BB, M, F, D)                                                                                      \
    k_cheb_mx<BB, M, F, D><<<grid, block, 0, st>>>(td.nb, td.Rp, c0, pr.rowptr.get(), pr.colidx.get(), Sv, y,   \
                                                   f, yio, Y, r, skip, it, a, b, partial, dpart, dot_active_only)
#define GSC_MX_F(BB, M)                                                              \
    if (fin == 0) { GSC_MX(BB, M, 0, false); }                                       \
    else if (fin == 1) { if (dot) GSC_MX(BB, M, 1, true); else GSC_MX(BB, M, 1, false); } \
    else { if (dot) GSC_MX(BB, M, 2, true); else GSC_MX(BB, M, 2, false); }
#define GSC_MX_B(BB) \
    if (mode == 0) { GSC_MX_F(BB, 0) } else if (mode == 1) { GSC_MX_F(BB, 1) } else { GSC_MX_F(BB, 2) }
    if (pr.B == 4) { GSC_MX_B(4) } else { GSC_MX_B(6) }
#undef GSC_MX_B
#undef GSC_MX_F
#undef GSC_MX
    GSC_HIP(hipGetLastError());
}

void launch_mx_resid(hipStream_t st, const Pair &pr, const TileDims &td, int col0, int ncols, const double *Sv,
                     const c128 *Y, const c128 *r, c64 *f, const int *skip, double *partial) {
    GSC_REQUIRE(col0 % 64 == 0 && ncols % 64 == 0 && ncols > 0 && col0 + ncols <= td.Rp,
                "Chebyshev column block outside the tile");
    dim3 grid(ncols / 64, td.Gs), block(kBlock);
    if (pr.B == 4)
        k_mx_resid<4><<<grid, block, 0, st>>>(td.nb, td.Rp, col0, pr.rowptr.get(), pr.colidx.get(), Sv, Y, r, f,
                                              skip, partial);
    else
        k_mx_resid<6><<<grid, block, 0, st>>>(td.nb, td.Rp, col0, pr.rowptr.get(), pr.colidx.get(), Sv, Y, r, f,
                                              skip, partial);
    GSC_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ launchers
// Row-group geometry of the product kernels (td.Gs row groups; every
// reduction of their partials uses td.Gs).  One block row per wave whenever
// the launch stays within 16384 workgroups: the rows a sweep keeps in flight
// then span few x-planes, whose halo fits L2, and no wave takes a second row
// while most take one (with 4096 groups over 4760 row slots, a 64-column
// launch on N = 76152 took 28 % longer than with one row each).  Wider
// launches keep about 4096 workgroups, at least 256 groups when there are
// more than 8 column chunks (an XCD would otherwise run the groups of
// several chunks at once, each with its own x window), and the groups are
// sized so that every wave takes the same number of rows.
void set_spmm_geometry(TileDims &td, const Pair &pr) {
    (void)pr;
    const int w = td.cb > 0 && td.cb < td.Rp ? td.cb : td.Rp;   // width of a Chebyshev launch
    const int chunks = std::max(1, w / 64);
    const int64_t slots = std::max<int64_t>(1, (td.nb + 3) / 4);   // groups for one row per wave
    int64_t g;
    if (chunks * slots <= 16384) {
        g = slots;
    } else {
        int64_t g0 = std::max(1, 4096 / chunks);
        if (chunks > 8) g0 = std::max<int64_t>(g0, 256);
        g0 = std::min(g0, slots);
        const int64_t passes = (slots + g0 - 1) / g0;
        g = (slots + passes - 1) / passes;
    }
    td.Gs = static_cast<int>((std::min<int64_t>(g, 65528) + 7) / 8 * 8);
}

template <typename T>
void launch_spmm_seed(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const T *Hv,
                      const cpx<T> *p, cpx<T> *q, const c128 *z, const int *seed, const int *skip,
                      c128 *partial) {
    dim3 grid(td.Rp / 64, td.Gs), block(kBlock);
    if (pr.B == 4)
        k_spmm_seed<T, 4><<<grid, block, 0, st>>>(td.nb, td.Rp, pr.rowptr.get(), pr.colidx.get(),
                                                  Sv, Hv, p, q, z, seed, skip, partial);
    else
        k_spmm_seed<T, 6><<<grid, block, 0, st>>>(td.nb, td.Rp, pr.rowptr.get(), pr.colidx.get(),
                                                  Sv, Hv, p, q, z, seed, skip, partial);
    GSC_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_S(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const cpx<T> *d,
                   cpx<T> *w, const int *skip, double *partial) {
    dim3 grid(td.Rp / 64, td.Gs), block(kBlock);
    if (pr.B == 4)
        k_spmm_S<T, 4><<<grid, block, 0, st>>>(td.nb, td.Rp, pr.rowptr.get(), pr.colidx.get(), Sv,
                                               d, w, skip, partial);
    else
        k_spmm_S<T, 6><<<grid, block, 0, st>>>(td.nb, td.Rp, pr.rowptr.get(), pr.colidx.get(), Sv,
                                               d, w, skip, partial);
    GSC_HIP(hipGetLastError());
}

template void launch_spmm_seed<double>(hipStream_t, const Pair &, const TileDims &, const double *,
                                       const double *, const c128 *, c128 *, const c128 *, const int *,
                                       const int *, c128 *);
template void launch_spmm_seed<float>(hipStream_t, const Pair &, const TileDims &, const float *,
                                      const float *, const c64 *, c64 *, const c128 *, const int *,
                                      const int *, c128 *);
template void launch_spmm_S<double>(hipStream_t, const Pair &, const TileDims &, const double *,
                                    const c128 *, c128 *, const int *, double *);
template void launch_spmm_S<float>(hipStream_t, const Pair &, const TileDims &, const float *, const c64 *,
                                   c64 *, const int *, double *);

}  // namespace gsc
