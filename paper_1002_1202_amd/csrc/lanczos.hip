// Products of the generalised Lanczos step (Sec. 3.2, eq. 1.13): h = H u and
// s = S u in one gather pass.  s is formed afresh every step: propagating it
// by the three-term recursion instead would carry the inner solve's error
// through a recursion that amplifies it by about |a_n| / b_n per step.
//
// The Lanczos vectors are real (S, H and the start vectors e_j are real), so
// two processes share one complex column: process 2c in the real parts and
// process 2c + 1 in the imaginary parts of column c.  Every linear operation
// of the step (the product with H, the solve with S) acts on the two parts
// separately; only the dot products must be split, which this kernel does:
// per column it leaves the partial sums of u_re h_re, u_im h_im (a_n of the
// two processes) and |h|^2 (the scale of the inner solve's tolerance).
// Layout and block order are those of the row product kernels.
#include "spmm.h"

namespace gsc {

template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_lz_hprod(int nb, int Rp, int Gs,
                                                     const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ colidx, const T *__restrict__ Hv,
                                                     const T *__restrict__ Sv, const cpx<T> *__restrict__ u,
                                                     cpx<T> *__restrict__ h, cpx<T> *__restrict__ su,
                                                     const int *__restrict__ skip, double *__restrict__ part) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = cx * 64 + lane;
    const bool act = !skip[col];
    double dre = 0.0, dim = 0.0, nrm = 0.0;
    // rows of this wave: every row group takes one row per wave per step, so
    // the groups advance together (step i covers rows [i*4*Gs, (i+1)*4*Gs))
    // and the rows in flight on an XCD stay within one window, however many
    // rows a group holds
    const int row_step = kWavesPerBlock * Gs;
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            cpx<T> acc[B], accs[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { acc[a] = {0, 0}; accs[a] = {0, 0}; own[a] = {0, 0}; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
            // loads of finished processes are masked off (their lines are not
            // fetched); their registers keep stale values that are never used
            cpx<T> xv[B];
#pragma unroll
            for (int c = 0; c < B; ++c) xv[c] = {0, 0};
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *hb = Hv + static_cast<size_t>(b) * B * B;
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                if (act) {
#pragma unroll
                    for (int c = 0; c < B; ++c) xv[c] = u[static_cast<size_t>(J * B + c) * Rp + col];
                }
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) own[c] = xv[c];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const T hv = hb[a * B + c], sv = sb[a * B + c];
                        acc[a].re = fma(hv, xv[c].re, acc[a].re);
                        acc[a].im = fma(hv, xv[c].im, acc[a].im);
                        accs[a].re = fma(sv, xv[c].re, accs[a].re);
                        accs[a].im = fma(sv, xv[c].im, accs[a].im);
                    }
                }
            }
            if (!act) continue;
#pragma unroll
            for (int a = 0; a < B; ++a) {
                h[static_cast<size_t>(I * B + a) * Rp + col] = acc[a];
                su[static_cast<size_t>(I * B + a) * Rp + col] = accs[a];
                dre += static_cast<double>(own[a].re) * acc[a].re;
                dim += static_cast<double>(own[a].im) * acc[a].im;
                nrm += static_cast<double>(acc[a].re) * acc[a].re + static_cast<double>(acc[a].im) * acc[a].im;
            }
        }
    }
    __shared__ double red[3][kWavesPerBlock][64];
    red[0][wv][lane] = dre;
    red[1][wv][lane] = dim;
    red[2][wv][lane] = nrm;
    __syncthreads();
    if (threadIdx.x < 64) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < kWavesPerBlock; ++k) t += red[q][k][lane];
            part[(static_cast<size_t>(q) * Gs + g) * Rp + col] = t;
        }
    }
}

template <typename T>
void launch_lz_hprod(hipStream_t st, const Pair &pr, const TileDims &td, const T *Hv, const T *Sv, const cpx<T> *u,
                     cpx<T> *h, cpx<T> *su, const int *skip, double *part) {
    dim3 grid(td.Rp / 64, td.Gs), block(kBlock);
    if (pr.B == 4)
        k_lz_hprod<T, 4><<<grid, block, 0, st>>>(static_cast<int>(pr.nb), td.Rp, td.Gs, pr.rowptr.get(),
                                                 pr.colidx.get(), Hv, Sv, u, h, su, skip, part);
    else
        k_lz_hprod<T, 6><<<grid, block, 0, st>>>(static_cast<int>(pr.nb), td.Rp, td.Gs, pr.rowptr.get(),
                                                 pr.colidx.get(), Hv, Sv, u, h, su, skip, part);
    GSC_HIP(hipGetLastError());
}

template void launch_lz_hprod<double>(hipStream_t, const Pair &, const TileDims &, const double *, const double *,
                                      const c128 *, c128 *, c128 *, const int *, double *);
template void launch_lz_hprod<float>(hipStream_t, const Pair &, const TileDims &, const float *, const float *,
                                     const c64 *, c64 *, c64 *, const int *, double *);

}  // namespace gsc
