// Gradient of a charge-dependent loss L = sum_r qbar_r q_{a_r} (Mulliken
// charges, Sec. 2.2) on the stored entries of H and S:
//   dL/dH_bc = -(2/pi) sum_k w_k sum_r qbar_r Im[lam_b x_c],
//   dL/dS_bc = -(2/pi) sum_k w_k sum_r qbar_r Im[delta_{a_r b} x_c - z_k lam_b x_c],
// with x = G_k e_a (the Green's-function column) and lam = G_k S e_a (the
// same shifted solver on the right-hand side S e_a); G is complex symmetric,
// so (S G)_ab = lam_b.  One workgroup per stored block, threads over the
// (shift, rhs) pairs of the tile, register accumulators, then a reduction.
#include "kernels.h"

namespace gsc {

namespace {

// columns S e_a (= rows, S is symmetric) of the tile's orbitals: out [R][N]
template <int B>
__global__ __launch_bounds__(kBlock) void k_s_columns(int N, const int32_t *rowptr, const int32_t *colidx,
                                                      const double *S, const int64_t *orbs, c128 *out) {
    const int r = blockIdx.x;
    const int64_t a = orbs[r];
    const int I = static_cast<int>(a / B), al = static_cast<int>(a % B);
    c128 *o = out + static_cast<size_t>(r) * N;
    for (int b = rowptr[I] + threadIdx.x; b < rowptr[I + 1]; b += kBlock) {
        const int J = colidx[b];
#pragma unroll
        for (int c = 0; c < B; ++c) o[J * B + c] = c128{S[(static_cast<size_t>(b) * B + al) * B + c], 0.0};
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    return v;
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_charge_vjp(int N, int K, int R, const int32_t *brow, const int32_t *colidx,
                                                       const c128 *X, const c128 *Lm, const c128 *z, const double *w,
                                                       const double *qbar, const int64_t *orbs, double *dH,
                                                       double *dS) {
    const int b = blockIdx.x;
    const int I = brow[b], J = colidx[b];
    double aH[B][B], aS[B][B];
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j) { aH[i][j] = 0.0; aS[i][j] = 0.0; }
    const int KR = K * R;
    for (int kr = threadIdx.x; kr < KR; kr += kBlock) {
        const int k = kr / R, r = kr % R;
        const double cw = w[k] * qbar[r];
        const c128 zk = z[k];
        const int64_t a = orbs[r];
        const c128 *lv = Lm + static_cast<size_t>(kr) * N + static_cast<size_t>(I) * B;
        const c128 *xv = X + static_cast<size_t>(kr) * N + static_cast<size_t>(J) * B;
        c128 l[B], x[B];
#pragma unroll
        for (int i = 0; i < B; ++i) { l[i] = lv[i]; x[i] = xv[i]; }
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const bool diag = static_cast<int64_t>(I) * B + i == a;
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const c128 p = l[i] * x[j];
                aH[i][j] += cw * p.im;
                // Im(z p) = z.re p.im + z.im p.re
                aS[i][j] += cw * ((diag ? x[j].im : 0.0) - (zk.re * p.im + zk.im * p.re));
            }
        }
    }
    __shared__ double red[kWavesPerBlock][2 * B * B];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const double h = wave_sum(aH[i][j]), s = wave_sum(aS[i][j]);
            if (lane == 0) {
                red[wv][i * B + j] = h;
                red[wv][B * B + i * B + j] = s;
            }
        }
    __syncthreads();
    const double f = -2.0 / 3.14159265358979323846;
    for (int t = threadIdx.x; t < 2 * B * B; t += kBlock) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q) v += red[q][t];
        if (t < B * B) dH[static_cast<size_t>(b) * B * B + t] += f * v;
        else dS[static_cast<size_t>(b) * B * B + t - B * B] += f * v;
    }
}

}  // namespace

void launch_s_columns(hipStream_t st, const Pair &p, int R, const int64_t *orbs, c128 *out) {
    GSC_HIP(hipMemsetAsync(out, 0, static_cast<size_t>(R) * p.n * sizeof(c128), st));
    if (p.B == 4)
        k_s_columns<4><<<R, kBlock, 0, st>>>(static_cast<int>(p.n), p.rowptr.get(), p.colidx.get(), p.S.get(), orbs,
                                             out);
    else
        k_s_columns<6><<<R, kBlock, 0, st>>>(static_cast<int>(p.n), p.rowptr.get(), p.colidx.get(), p.S.get(), orbs,
                                             out);
    GSC_HIP(hipGetLastError());
}

void launch_charge_vjp(hipStream_t st, const Pair &p, int K, int R, const c128 *X, const c128 *Lm, const c128 *z,
                       const double *w, const double *qbar, const int64_t *orbs, double *dH, double *dS) {
    const unsigned grid = static_cast<unsigned>(p.nnzb);
    if (p.B == 4)
        k_charge_vjp<4><<<grid, kBlock, 0, st>>>(static_cast<int>(p.n), K, R, p.brow.get(), p.colidx.get(), X, Lm, z,
                                                 w, qbar, orbs, dH, dS);
    else
        k_charge_vjp<6><<<grid, kBlock, 0, st>>>(static_cast<int>(p.n), K, R, p.brow.get(), p.colidx.get(), X, Lm, z,
                                                 w, qbar, orbs, dH, dS);
    GSC_HIP(hipGetLastError());
}

}  // namespace gsc
