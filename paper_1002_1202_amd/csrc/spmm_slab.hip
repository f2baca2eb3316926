// Slab variants of the gathered products (S, H times many right-hand sides).
//
// A wave covers one block row I and a slab of CW right-hand sides; lane
// (a, c) computes orbital row I*B + a for column slab*CW + c, so the gathered
// x rows of a slab are CW*16 bytes (FP64) per orbital.  Blocks are ordered
// so that consecutive workgroups of one XCD walk the block rows of one slab
// in order: the halo of neighbour blocks (second shell) that a sweep keeps
// live is then a few MB and stays in that XCD's L2, instead of every XCD
// fetching the x rows of its own row range plus a halo as large as the range.
// The per-lane matrix row (B values) is the same for the CW lanes of an
// orbital row and is served as one broadcast per wave.
#include "spmm.h"

namespace gsc {

template <int B> struct Slab { static constexpr int CW = B == 4 ? 16 : 10; };

// slab index and row group of this workgroup; XCD x (= linear id mod 8)
// receives the slabs congruent to x and all their row groups in order
__device__ inline void slab_map(int nsl, int G, int &slab, int &g) {
    if (gridDim.x == 8) {
        slab = blockIdx.x + 8 * (blockIdx.y / G);
        g = blockIdx.y % G;
    } else {
        slab = blockIdx.x;
        g = blockIdx.y;
    }
    (void)nsl;
}

// sum over the lanes of one column (the B orbital rows) and over the 4 waves
template <typename V, int CW>
__device__ inline void slab_partial(V v, V *partial, int g, int Rp, int slab) {
    __shared__ V red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < CW) {
        V s = red[threadIdx.x];
        for (int w = 0; w < kWavesPerBlock; ++w)
            for (int a = 0; a * CW + static_cast<int>(threadIdx.x) < 64; ++a)
                if (w != 0 || a != 0) s = s + red[w * 64 + a * CW + threadIdx.x];
        const int col = slab * CW + threadIdx.x;
        if (col < Rp) partial[static_cast<size_t>(g) * Rp + col] = s;
    }
}

// gather of one block row: acc = sum_J M[I, J] row a times x_J (lanes of a
// slab), own = x of the diagonal block at orbital a
template <typename T, int B, bool TWO>
__device__ inline void slab_row(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                const T *__restrict__ M1, const T *__restrict__ M2, const cpx<T> *__restrict__ x,
                                int I, int a, int Rp, int col, bool act, cpx<T> &acc1, cpx<T> &acc2,
                                cpx<T> &own) {
    const int b0 = rowptr[I], b1 = rowptr[I + 1];
#pragma unroll 2
    for (int b = b0; b < b1; ++b) {
        const int J = colidx[b];
        cpx<T> xv[B];
        T m1[B], m2[B];
#pragma unroll
        for (int c = 0; c < B; ++c) {
            xv[c] = act ? x[static_cast<size_t>(J * B + c) * Rp + col] : cpx<T>{0, 0};
            m1[c] = act ? M1[(static_cast<size_t>(b) * B + a) * B + c] : T(0);
            if (TWO) m2[c] = act ? M2[(static_cast<size_t>(b) * B + a) * B + c] : T(0);
        }
#pragma unroll
        for (int c = 0; c < B; ++c) {
            acc1.re = fma(m1[c], xv[c].re, acc1.re);
            acc1.im = fma(m1[c], xv[c].im, acc1.im);
            if (TWO) {
                acc2.re = fma(m2[c], xv[c].re, acc2.re);
                acc2.im = fma(m2[c], xv[c].im, acc2.im);
            }
        }
        if (J == I) {
#pragma unroll
            for (int c = 0; c < B; ++c)
                if (c == a) own = xv[c];
        }
    }
}

// q = zs_c S p - H p, partial p^T q
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_spmm_seed_slab(
    int nb, int Rp, int G, int nsl, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const T *__restrict__ Hv, const cpx<T> *__restrict__ p, cpx<T> *__restrict__ q,
    const c128 *__restrict__ z, const int *__restrict__ seed, const int *__restrict__ skip,
    c128 *__restrict__ partial) {
    constexpr int CW = Slab<B>::CW;
    int slab, g;
    slab_map(nsl, G, slab, g);
    const int lane = threadIdx.x & 63;
    const int a = lane / CW;
    const int col = slab * CW + lane % CW;
    const int I = g * kWavesPerBlock + wave_id();
    const bool act = a < B && col < Rp && I < nb && (skip == nullptr || !skip[col]);
    c128 dot{0, 0};
    if (__ballot(act) != 0) {
        cpx<T> aS{0, 0}, aH{0, 0}, own{0, 0};
        slab_row<T, B, true>(rowptr, colidx, Sv, Hv, p, I, a, Rp, col, act, aS, aH, own);
        if (act) {
            const c128 zs = z[seed[col]];
            const cpx<T> v = ccast<T>(zs) * aS - aH;
            q[static_cast<size_t>(I * B + a) * Rp + col] = v;
            dot = ccast<double>(own) * ccast<double>(v);
        }
    }
    slab_partial<c128, CW>(dot, partial, g, Rp, slab);
}

// w = S d, partial Re(d^H S d)
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_spmm_S_slab(
    int nb, int Rp, int G, int nsl, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const cpx<T> *__restrict__ d, cpx<T> *__restrict__ wout,
    const int *__restrict__ skip, double *__restrict__ partial) {
    constexpr int CW = Slab<B>::CW;
    int slab, g;
    slab_map(nsl, G, slab, g);
    const int lane = threadIdx.x & 63;
    const int a = lane / CW;
    const int col = slab * CW + lane % CW;
    const int I = g * kWavesPerBlock + wave_id();
    const bool act = a < B && col < Rp && I < nb && !skip[col];
    double dot = 0.0;
    if (__ballot(act) != 0) {
        cpx<T> aS{0, 0}, unused{0, 0}, own{0, 0};
        slab_row<T, B, false>(rowptr, colidx, Sv, Sv, d, I, a, Rp, col, act, aS, unused, own);
        if (act) {
            wout[static_cast<size_t>(I * B + a) * Rp + col] = aS;
            dot = static_cast<double>(own.re) * aS.re + static_cast<double>(own.im) * aS.im;
        }
    }
    slab_partial<double, CW>(dot, partial, g, Rp, slab);
}

// Chebyshev step fused with the product (see k_cheb_step)
template <typename T, int B, int MODE>
__global__ __launch_bounds__(kBlock) void k_cheb_slab(
    int nb, int Rp, int G, int nsl, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ Sv, const cpx<T> *__restrict__ y, const cpx<T> *__restrict__ r,
    cpx<T> *__restrict__ yio, const int *__restrict__ skip, T inv_theta, T c1, T c2,
    double *__restrict__ partial) {
    constexpr int CW = Slab<B>::CW;
    int slab, g;
    slab_map(nsl, G, slab, g);
    const int lane = threadIdx.x & 63;
    const int a = lane / CW;
    const int col = slab * CW + lane % CW;
    const int I = g * kWavesPerBlock + wave_id();
    const bool act = a < B && col < Rp && I < nb && !skip[col];
    double acc2 = 0.0;
    if (__ballot(act) != 0) {
        cpx<T> aS{0, 0}, unused{0, 0}, own{0, 0};
        slab_row<T, B, false>(rowptr, colidx, Sv, Sv, MODE == 0 ? r : y, I, a, Rp, col, act, aS, unused, own);
        if (act)
            acc2 = cheb_update<T, MODE, false>(own, aS, r, yio, static_cast<size_t>(I * B + a) * Rp + col, inv_theta,
                                               c1, c2);
    }
    slab_partial<double, CW>(acc2, partial, g, Rp, slab);
}

// ------------------------------------------------------------------ launchers
int slab_groups(int nb) { return (nb + kWavesPerBlock - 1) / kWavesPerBlock; }

static dim3 slab_grid(int B, int Rp, int G) {
    const int CW = B == 4 ? Slab<4>::CW : Slab<6>::CW;
    const int nsl = (Rp + CW - 1) / CW;
    if (nsl % 8 == 0) return dim3(8, G * (nsl / 8));
    return dim3(nsl, G);
}

template <typename T>
void launch_spmm_seed_slab(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const T *Hv,
                           const cpx<T> *p, cpx<T> *q, const c128 *z, const int *seed, const int *skip,
                           c128 *partial) {
    const dim3 grid = slab_grid(pr.B, td.Rp, td.Gs);
    const int nsl = pr.B == 4 ? (td.Rp + 15) / 16 : (td.Rp + 9) / 10;
    if (pr.B == 4)
        k_spmm_seed_slab<T, 4><<<grid, kBlock, 0, st>>>(td.nb, td.Rp, td.Gs, nsl, pr.rowptr.get(), pr.colidx.get(),
                                                        Sv, Hv, p, q, z, seed, skip, partial);
    else
        k_spmm_seed_slab<T, 6><<<grid, kBlock, 0, st>>>(td.nb, td.Rp, td.Gs, nsl, pr.rowptr.get(), pr.colidx.get(),
                                                        Sv, Hv, p, q, z, seed, skip, partial);
    GSC_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_S_slab(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const cpx<T> *d, cpx<T> *w,
                        const int *skip, double *partial) {
    const dim3 grid = slab_grid(pr.B, td.Rp, td.Gs);
    const int nsl = pr.B == 4 ? (td.Rp + 15) / 16 : (td.Rp + 9) / 10;
    if (pr.B == 4)
        k_spmm_S_slab<T, 4><<<grid, kBlock, 0, st>>>(td.nb, td.Rp, td.Gs, nsl, pr.rowptr.get(), pr.colidx.get(), Sv,
                                                     d, w, skip, partial);
    else
        k_spmm_S_slab<T, 6><<<grid, kBlock, 0, st>>>(td.nb, td.Rp, td.Gs, nsl, pr.rowptr.get(), pr.colidx.get(), Sv,
                                                     d, w, skip, partial);
    GSC_HIP(hipGetLastError());
}

template <typename T>
void launch_cheb_slab(hipStream_t st, const Pair &pr, const TileDims &td, int mode, const T *Sv, const cpx<T> *y,
                      const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta, double c1, double c2,
                      double *partial) {
    const dim3 grid = slab_grid(pr.B, td.Rp, td.Gs);
    const int nsl = pr.B == 4 ? (td.Rp + 15) / 16 : (td.Rp + 9) / 10;
    const T it = static_cast<T>(inv_theta), a = static_cast<T>(c1), b = static_cast<T>(c2);
#define GSC_CS(BB, M)                                                                                           \
    k_cheb_slab<T, BB, M><<<grid, kBlock, 0, st>>>(td.nb, td.Rp, td.Gs, nsl, pr.rowptr.get(), pr.colidx.get(), Sv, \
                                                   y, r, yio, skip, it, a, b, partial)
#define GSC_CS_B(BB) \
    if (mode == 0) GSC_CS(BB, 0); else if (mode == 1) GSC_CS(BB, 1); else GSC_CS(BB, 2);
    if (pr.B == 4) { GSC_CS_B(4) } else { GSC_CS_B(6) }
#undef GSC_CS_B
#undef GSC_CS
    GSC_HIP(hipGetLastError());
}

#define GSC_INST(T)                                                                                                 \
    template void launch_spmm_seed_slab<T>(hipStream_t, const Pair &, const TileDims &, const T *, const T *,       \
                                           const cpx<T> *, cpx<T> *, const c128 *, const int *, const int *, c128 *); \
    template void launch_spmm_S_slab<T>(hipStream_t, const Pair &, const TileDims &, const T *, const cpx<T> *,     \
                                        cpx<T> *, const int *, double *);                                           \
    template void launch_cheb_slab<T>(hipStream_t, const Pair &, const TileDims &, int, const T *, const cpx<T> *, \
                                      const cpx<T> *, cpx<T> *, const int *, double, double, double, double *);
GSC_INST(double)
GSC_INST(float)
#undef GSC_INST

}  // namespace gsc
