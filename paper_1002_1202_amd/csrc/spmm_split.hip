// Split-orbital variant of the Chebyshev-fused S product.
//
// A wave owns one block row and 32 consecutive right-hand sides; its two
// half-waves take the two halves of the gathered block's orbital index (B/2
// orbital rows each), so every load is still one 16-byte (FP64) element
// per lane and one coalesced 512 B segment per orbital row per half.  The
// S entries a half needs are selected per lane from the wave-uniform block,
// and the two halves' partial sums are added with one cross-lane swap per
// block row.  With 256 columns there are 8 stripes: XCD x owns stripe x and
// sweeps every block row, so the x halo its resident waves keep live is half
// that of a 64-column stripe and fits its L2.
#include "spmm.h"

namespace gsc {

template <typename T>
__device__ inline cpx<T> swap_halves(cpx<T> v) {
    return {__shfl_xor(v.re, 32), __shfl_xor(v.im, 32)};
}

template <typename T, int B, int MODE, bool NT>
__global__ __launch_bounds__(kBlock) void k_cheb_split(
    int nb, int Rp, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const cpx<T> *__restrict__ y, const cpx<T> *__restrict__ r, cpx<T> *__restrict__ yio,
    const int *__restrict__ skip, T inv_theta, T c1, T c2, double *__restrict__ partial) {
    constexpr int H = B / 2;
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const bool hi = lane >= 32;
    const int h0 = hi ? H : 0;       // first orbital of this half
    const int wv = wave_id();
    const int col = cx * 32 + (lane & 31);
    const bool act = !skip[col];
    double acc2 = 0.0;
    // rows of this wave: every row group takes one row per wave per step, so
    // the groups advance together (step i covers rows [i*4*Gs, (i+1)*4*Gs))
    const int row_step = kWavesPerBlock * static_cast<int>(gridDim.y);
    const cpx<T> *x = MODE == 0 ? r : y;
    if (__ballot(act) != 0) {
        for (int I = kWavesPerBlock * g + wv; I < nb; I += row_step) {
            cpx<T> aS[B], own[H];
#pragma unroll
            for (int a = 0; a < B; ++a) aS[a] = {0, 0};
#pragma unroll
            for (int c = 0; c < H; ++c) own[c] = {0, 0};
            const int b0 = rowptr[I], b1 = rowptr[I + 1];
#pragma unroll 2
            for (int b = b0; b < b1; ++b) {
                const int J = colidx[b];
                const T *sb = Sv + static_cast<size_t>(b) * B * B;
                cpx<T> xv[H];
#pragma unroll
                for (int c = 0; c < H; ++c)
                    xv[c] = x[static_cast<size_t>(J * B + h0 + c) * Rp + col];
                if (J == I) {
#pragma unroll
                    for (int c = 0; c < H; ++c) own[c] = xv[c];
                }
#pragma unroll
                for (int a = 0; a < B; ++a) {
#pragma unroll
                    for (int c = 0; c < H; ++c) {
                        const T s_lo = sb[a * B + c], s_hi = sb[a * B + H + c];
                        const T sv = hi ? s_hi : s_lo;
                        aS[a].re = fma(sv, xv[c].re, aS[a].re);
                        aS[a].im = fma(sv, xv[c].im, aS[a].im);
                    }
                }
            }
            // full row sums; half h finalizes its own orbital rows h0 + c
            cpx<T> Sx[H];
#pragma unroll
            for (int c = 0; c < H; ++c) {
                const cpx<T> mine_lo = aS[c], mine_hi = aS[H + c];
                // the other half needs the rows this half does not finalize
                const cpx<T> give = hi ? mine_lo : mine_hi;
                const cpx<T> got = swap_halves(give);
                const cpx<T> keep = hi ? mine_hi : mine_lo;
                Sx[c] = keep + got;
            }
            if (!act) continue;
#pragma unroll
            for (int c = 0; c < H; ++c)
                acc2 += cheb_update<T, MODE, NT>(own[c], Sx[c], r, yio,
                                                 static_cast<size_t>(I * B + h0 + c) * Rp + col, inv_theta, c1, c2);
        }
    }
    // the two halves of a column and the 4 waves add into one partial
    __shared__ double red[kWavesPerBlock][64];
    red[wv][lane] = acc2;
    __syncthreads();
    if (threadIdx.x < 32) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) t += red[k][threadIdx.x] + red[k][threadIdx.x + 32];
        partial[static_cast<size_t>(g) * Rp + cx * 32 + threadIdx.x] = t;
    }
}

template <typename T>
void launch_cheb_split(hipStream_t st, const Pair &pr, const TileDims &td, int mode, const T *Sv, const cpx<T> *y,
                       const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta, double c1, double c2,
                       double *partial) {
    dim3 grid(td.Rp / 32, td.Gs), block(kBlock);
    const T it = static_cast<T>(inv_theta), a = static_cast<T>(c1), b = static_cast<T>(c2);
#define GSC_CHEB_SP(BB, M, N)                                                                                       \
    k_cheb_split<T, BB, M, N><<<grid, block, 0, st>>>(td.nb, td.Rp, pr.rowptr.get(), pr.colidx.get(), Sv, y, \
                                                      r, yio, skip, it, a, b, partial)
#define GSC_CHEB_SP_N(BB, M) \
    if (td.nt) GSC_CHEB_SP(BB, M, true); else GSC_CHEB_SP(BB, M, false);
#define GSC_CHEB_SP_B(BB) \
    if (mode == 0) { GSC_CHEB_SP_N(BB, 0) } else if (mode == 1) { GSC_CHEB_SP_N(BB, 1) } else { GSC_CHEB_SP_N(BB, 2) }
    if (pr.B == 4) { GSC_CHEB_SP_B(4) } else { GSC_CHEB_SP_B(6) }
#undef GSC_CHEB_SP_B
#undef GSC_CHEB_SP_N
#undef GSC_CHEB_SP
    GSC_HIP(hipGetLastError());
}

template void launch_cheb_split<double>(hipStream_t, const Pair &, const TileDims &, int, const double *,
                                        const c128 *, const c128 *, c128 *, const int *, double, double, double,
                                        double *);
template void launch_cheb_split<float>(hipStream_t, const Pair &, const TileDims &, int, const float *, const c64 *,
                                       const c64 *, c64 *, const int *, double, double, double, double *);

}  // namespace gsc
