// Cluster variant of the Chebyshev-fused S product.
//
// A wave owns one cluster of C consecutive block rows (C = 8 for B = 4, one
// diamond cell) and 64 right-hand sides, and walks the cluster's union of
// column blocks once: each x row of the union is loaded once per cluster
// instead of once per block row that references it (56 loads instead of 136
// per silicon cell), and applied to every row of the cluster that stores a
// block in that column.  The walk is driven by the packed list of the pair's
// clusters (column | row mask << 24) and by a copy of S whose blocks are
// permuted into walk order, so no lookup depends on another load; the row
// loop is unrolled with wave-uniform branches so that the C x B complex
// accumulators stay in registers.
#include "spmm.h"

namespace gsc {

// dst block k = src block perm[k] (walk-ordered copy of the block values)
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_permute_blocks(int64_t nnzb, const int32_t *__restrict__ perm,
                                                           const T *__restrict__ src, T *__restrict__ dst) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= nnzb * B * B) return;
    const int64_t k = t / (B * B), o = t % (B * B);
    dst[t] = src[static_cast<int64_t>(perm[k]) * B * B + o];
}

template <typename T, int B, int C, int MODE>
__global__ __launch_bounds__(kBlock) void k_cheb_cl(
    int nb, int nc, int Rp, const int32_t *__restrict__ ptr, const int32_t *__restrict__ pack,
    const int32_t *__restrict__ sptr, const T *__restrict__ Scl, const cpx<T> *__restrict__ y,
    const cpx<T> *__restrict__ r, cpx<T> *__restrict__ yio, const int *__restrict__ skip, T inv_theta, T c1, T c2,
    double *__restrict__ partial) {
    int cx, g;
    xcd_remap_chunks(cx, g);
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int col = cx * 64 + lane;
    const bool act = !skip[col];
    const int c = g * kWavesPerBlock + wv;
    const cpx<T> *x = MODE == 0 ? r : y;
    double acc2 = 0.0;
    if (c < nc && __ballot(act) != 0) {
        cpx<T> acc[C][B];
#pragma unroll
        for (int i = 0; i < C; ++i)
#pragma unroll
            for (int a = 0; a < B; ++a) acc[i][a] = {0, 0};
        const int u0 = ptr[c], u1 = ptr[c + 1];
        const T *sb = Scl + static_cast<size_t>(sptr[c]) * B * B;
        for (int u = u0; u < u1; ++u) {
            const uint32_t pk = static_cast<uint32_t>(pack[u]);
            const int J = static_cast<int>(pk & 0xffffffu);
            const uint32_t mask = pk >> 24;
            cpx<T> xv[B];
#pragma unroll
            for (int cc = 0; cc < B; ++cc)
                xv[cc] = x[static_cast<size_t>(J * B + cc) * Rp + col];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (mask & (1u << i)) {
#pragma unroll
                    for (int a = 0; a < B; ++a) {
#pragma unroll
                        for (int cc = 0; cc < B; ++cc) {
                            const T sv = sb[a * B + cc];
                            acc[i][a].re = fma(sv, xv[cc].re, acc[i][a].re);
                            acc[i][a].im = fma(sv, xv[cc].im, acc[i][a].im);
                        }
                    }
                    sb += B * B;
                }
            }
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const int I = c * C + i;
                if (I < nb) {
#pragma unroll
                    for (int a = 0; a < B; ++a) {
                        const size_t e = static_cast<size_t>(I * B + a) * Rp + col;
                        acc2 += cheb_update<T, MODE, false>(x[e], acc[i][a], r, yio, e, inv_theta, c1, c2);
                    }
                }
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

template <typename T>
void launch_permute_blocks(hipStream_t st, const Pair &pr, const T *src, T *dst) {
    GSC_REQUIRE(pr.cl.perm.get() != nullptr, "cluster walk lists are not available for this pair");
    const int64_t n = pr.nnzb * pr.B * pr.B;
    const unsigned grid = static_cast<unsigned>((n + kBlock - 1) / kBlock);
    if (pr.B == 4) k_permute_blocks<T, 4><<<grid, kBlock, 0, st>>>(pr.nnzb, pr.cl.perm.get(), src, dst);
    else k_permute_blocks<T, 6><<<grid, kBlock, 0, st>>>(pr.nnzb, pr.cl.perm.get(), src, dst);
    GSC_HIP(hipGetLastError());
}

template <typename T>
void launch_cheb_cl(hipStream_t st, const Pair &pr, const TileDims &td, int mode, const T *Scl, const cpx<T> *y,
                    const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta, double c1, double c2,
                    double *partial) {
    GSC_REQUIRE(pr.cl.pack.get() != nullptr, "cluster walk lists are not available for this pair");
    dim3 grid(td.Rp / 64, td.Gs), block(kBlock);
    const T it = static_cast<T>(inv_theta), a = static_cast<T>(c1), b = static_cast<T>(c2);
#define GSC_CCL(BB, CC, M)                                                                                     \
    k_cheb_cl<T, BB, CC, M><<<grid, block, 0, st>>>(static_cast<int>(pr.nb), pr.cl.nc, td.Rp, pr.cl.ptr.get(), \
                                                    pr.cl.pack.get(), pr.cl.sptr.get(), Scl, y, r, yio, skip, it, \
                                                    a, b, partial)
#define GSC_CCL_B(BB, CC) \
    if (mode == 0) GSC_CCL(BB, CC, 0); else if (mode == 1) GSC_CCL(BB, CC, 1); else GSC_CCL(BB, CC, 2);
    if (pr.B == 4) {
        GSC_REQUIRE(pr.cl.C == 8, "cluster size mismatch");
        GSC_CCL_B(4, 8)
    } else {
        GSC_REQUIRE(pr.cl.C == 4, "cluster size mismatch");
        GSC_CCL_B(6, 4)
    }
#undef GSC_CCL_B
#undef GSC_CCL
    GSC_HIP(hipGetLastError());
}

template void launch_permute_blocks<double>(hipStream_t, const Pair &, const double *, double *);
template void launch_permute_blocks<float>(hipStream_t, const Pair &, const float *, float *);
template void launch_cheb_cl<double>(hipStream_t, const Pair &, const TileDims &, int, const double *, const c128 *,
                                     const c128 *, c128 *, const int *, double, double, double, double *);
template void launch_cheb_cl<float>(hipStream_t, const Pair &, const TileDims &, int, const float *, const c64 *,
                                    const c64 *, c64 *, const int *, double, double, double, double *);

}  // namespace gsc
