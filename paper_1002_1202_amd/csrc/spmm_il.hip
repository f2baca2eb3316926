// Interleaved-real variant of the Chebyshev-fused S product.
//
// A complex vector of Rp columns is read as a real array of 2 Rp values per
// orbital row (re, im interleaved).  One wave owns 64 consecutive reals (32
// complex columns) and one block row at a time: since S is real, every real
// lane is an independent real product with the same wave-uniform S block,
// so the gathered loads stay one coalesced 512 B (FP64) segment per orbital
// row with no redundant lanes, and the Chebyshev update acts componentwise.
// With 256 columns there are 8 such stripes: XCD x owns stripe x and sweeps
// every block row in order, so the x halo that a sweep keeps live is half
// that of a 64-column stripe and stays in that XCD's L2.  With NT the
// streamed operands (r, d and the written iterate) bypass L2 retention so
// that they do not evict the halo.
#include "spmm.h"

namespace gsc {

template <typename T, int B, bool FIRST, bool NT>
__global__ __launch_bounds__(kBlock) void k_cheb_il(
    int nb, int Rp, int Lb, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const T *__restrict__ y, const T *__restrict__ r, T *__restrict__ dvec,
    T *__restrict__ ynext, const int *__restrict__ skip, T inv_theta, T c1, T c2,
    double *__restrict__ partial) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int e0 = cx * 64 + lane;  // real index inside an orbital row
    const size_t ld = 2 * static_cast<size_t>(Rp);
    const bool act = !skip[e0 >> 1];
    double acc2 = 0.0;
    const int I0 = g * Lb;
    const int I1 = min(nb, I0 + Lb);
    const T *x = FIRST ? r : y;
    if (__ballot(act) != 0) {
        for (int I = I0 + wv; I < I1; I += kWavesPerBlock) {
            T aS[B], own[B];
#pragma unroll
            for (int a = 0; a < B; ++a) { aS[a] = 0; own[a] = 0; }
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                T xv[B];
#pragma unroll
                for (int c = 0; c < B; ++c) xv[c] = act ? x[static_cast<size_t>(J * B + c) * ld + e0] : T(0);
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < B; ++c) own[c] = xv[c];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < B; ++c) aS[a] = fma(sb[a * B + c], xv[c], aS[a]);
                }
            }
            if (!act) continue;
#pragma unroll
            for (int a = 0; a < B; ++a) {
                const size_t e = static_cast<size_t>(I * B + a) * ld + e0;
                T yk, dprev, Sy = aS[a];
                const T rv = FIRST ? own[a] : ld_stream<T, NT>(r + e);
                if (FIRST) {
                    yk = inv_theta * own[a];
                    dprev = yk;
                    Sy = inv_theta * Sy;
                } else {
                    yk = own[a];
                    dprev = ld_stream<T, NT>(dvec + e);
                }
                const T res = rv - Sy;
                const T dn = c1 * dprev + c2 * res;
                st_stream<T, NT>(dn, dvec + e);
                st_stream<T, NT>(yk + dn, ynext + e);
                acc2 += static_cast<double>(res) * res;
            }
        }
    }
    // the two lanes of a complex column and the 4 waves add into one partial
    __shared__ double red[kWavesPerBlock][64];
    red[wv][lane] = acc2;
    __syncthreads();
    if (threadIdx.x < 32) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) t += red[k][2 * threadIdx.x] + red[k][2 * threadIdx.x + 1];
        partial[static_cast<size_t>(g) * Rp + cx * 32 + threadIdx.x] = t;
    }
}

template <typename T>
void launch_cheb_il(hipStream_t st, const Pair &pr, const TileDims &td, bool first, const T *Sv, const cpx<T> *y,
                    const cpx<T> *r, cpx<T> *d, cpx<T> *ynext, const int *skip, double inv_theta, double c1,
                    double c2, double *partial) {
    dim3 grid(td.Rp / 32, td.Gs), block(kBlock);
    const T it = static_cast<T>(inv_theta), a = static_cast<T>(c1), b = static_cast<T>(c2);
    const T *yr = reinterpret_cast<const T *>(y);
    const T *rr = reinterpret_cast<const T *>(r);
    T *dr = reinterpret_cast<T *>(d);
    T *yn = reinterpret_cast<T *>(ynext);
#define GSC_CHEB_IL(BB, F, N)                                                                                    \
    k_cheb_il<T, BB, F, N><<<grid, block, 0, st>>>(td.nb, td.Rp, td.Lb, pr.rowptr.get(), pr.colidx.get(), Sv, yr, \
                                                   rr, dr, yn, skip, it, a, b, partial)
#define GSC_CHEB_IL_B(BB)                                          \
    if (first) { if (td.nt) GSC_CHEB_IL(BB, true, true); else GSC_CHEB_IL(BB, true, false); } \
    else { if (td.nt) GSC_CHEB_IL(BB, false, true); else GSC_CHEB_IL(BB, false, false); }
    if (pr.B == 4) { GSC_CHEB_IL_B(4) } else { GSC_CHEB_IL_B(6) }
#undef GSC_CHEB_IL_B
#undef GSC_CHEB_IL
    GSC_HIP(hipGetLastError());
}

template void launch_cheb_il<double>(hipStream_t, const Pair &, const TileDims &, bool, const double *, const c128 *,
                                     const c128 *, c128 *, c128 *, const int *, double, double, double, double *);
template void launch_cheb_il<float>(hipStream_t, const Pair &, const TileDims &, bool, const float *, const c64 *,
                                    const c64 *, c64 *, c64 *, const int *, double, double, double, double *);

}  // namespace gsc
