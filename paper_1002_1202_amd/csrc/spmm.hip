// Block-sparse products with H and S for many right-hand sides at once.
//
// One wave owns 64 consecutive columns and walks one block row at a time;
// the B x B blocks of S and H are wave-uniform (scalar loads), the gathered
// x rows are 64 contiguous complex values per orbital (one coalesced
// 1 KiB (FP64) transaction per orbital row).  No MFMA: per stored value the
// product does 2 (S only) or 4 (S and H) FMAs per complex column against
// >= 16 bytes of vector traffic, far below the FP64 ridge.
#include "spmm.h"

namespace gsc {

// q = zs_c * (S p) - H p for every active column c, plus the per-column
// unconjugated partial dot  sum_i p_i q_i  (the denominator of alpha,
// eq. CGp:r with the S-bilinear form) of this row group.
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_spmm_seed(
    int nb, int Rp, int Lb, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const T *__restrict__ Hv, const cpx<T> *__restrict__ p,
    cpx<T> *__restrict__ q, const c128 *__restrict__ z, const int *__restrict__ seed,
    const int *__restrict__ skip, c128 *__restrict__ partial) {
    int cx, g;
    xcd_remap(cx, g);
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int col = cx * 64 + lane;
    const bool act = skip == nullptr || !skip[col];
    c128 zs = act ? z[seed[col]] : c128{0, 0};
    const cpx<T> zt = ccast<T>(zs);
    c128 dot{0.0, 0.0};
    const int I0 = g * Lb;
    const int I1 = min(nb, I0 + Lb);
    if (__ballot(act) != 0) {
        for (int I = I0 + w; I < I1; I += kWavesPerBlock) {
            cpx<T> aS[B], aH[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = {0, 0}; aH[a] = {0, 0}; own[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                const T *hb = Hv + static_cast<size_t>(b) * B * B;
                cpx<T> x[B];
#pragma unroll
                for (int c = 0; c < B; ++c)
                    x[c] = act ? p[static_cast<size_t>(J * B + c) * Rp + col] : cpx<T>{0, 0};
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) own[c] = x[c];
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
#pragma unroll
            for (int a = 0; a < B; ++a) {
                const cpx<T> v = zt * aS[a] - aH[a];
                if (act) {
                    q[static_cast<size_t>(I * B + a) * Rp + col] = v;
                    dot = dot + ccast<double>(own[a]) * ccast<double>(v);
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
    int nb, int Rp, int Lb, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const cpx<T> *__restrict__ d, cpx<T> *__restrict__ wout,
    const int *__restrict__ skip, double *__restrict__ partial) {
    int cx, g;
    xcd_remap(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = cx * 64 + lane;
    const bool act = !skip[col];
    double dot = 0.0;
    const int I0 = g * Lb;
    const int I1 = min(nb, I0 + Lb);
    if (__ballot(act) != 0) {
        for (int I = I0 + wv; I < I1; I += kWavesPerBlock) {
            cpx<T> aS[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = {0, 0}; own[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                cpx<T> x[B];
#pragma unroll
                for (int c = 0; c < B; ++c)
                    x[c] = act ? d[static_cast<size_t>(J * B + c) * Rp + col] : cpx<T>{0, 0};
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

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_spmm_seed(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const T *Hv,
                      const cpx<T> *p, cpx<T> *q, const c128 *z, const int *seed, const int *skip,
                      c128 *partial) {
    dim3 grid(td.Rp / 64, td.Gs), block(kBlock);
    if (pr.B == 4)
        k_spmm_seed<T, 4><<<grid, block, 0, st>>>(td.nb, td.Rp, td.Lb, pr.rowptr.get(), pr.colidx.get(),
                                                  Sv, Hv, p, q, z, seed, skip, partial);
    else
        k_spmm_seed<T, 6><<<grid, block, 0, st>>>(td.nb, td.Rp, td.Lb, pr.rowptr.get(), pr.colidx.get(),
                                                  Sv, Hv, p, q, z, seed, skip, partial);
    GSC_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_S(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const cpx<T> *d,
                   cpx<T> *w, const int *skip, double *partial) {
    dim3 grid(td.Rp / 64, td.Gs), block(kBlock);
    if (pr.B == 4)
        k_spmm_S<T, 4><<<grid, block, 0, st>>>(td.nb, td.Rp, td.Lb, pr.rowptr.get(), pr.colidx.get(), Sv,
                                               d, w, skip, partial);
    else
        k_spmm_S<T, 6><<<grid, block, 0, st>>>(td.nb, td.Rp, td.Lb, pr.rowptr.get(), pr.colidx.get(), Sv,
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
