#pragma once
#include "kernels.h"

namespace gsc {

// variant 0: one block row per wave; 1: register-blocked clusters; 2: slabs;
// 3: split-orbital stripes of 32 columns for the Chebyshev step (the other
// products use the variant-0 kernels on the same row groups)
void set_spmm_geometry(TileDims &td, const Pair &pr, int variant);

template <typename T>
void launch_spmm_seed(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const T *Hv,
                      const cpx<T> *p, cpx<T> *q, const c128 *z, const int *seed, const int *skip,
                      c128 *partial);

template <typename T>
void launch_spmm_S(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const cpx<T> *d,
                   cpx<T> *w, const int *skip, double *partial);

template <typename T>
void launch_cheb_step(hipStream_t st, const Pair &pr, const TileDims &td, int mode, int col0, int ncols, const T *Sv,
                      const cpx<T> *y, const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta,
                      double c1, double c2, double *partial, c128 *dpart = nullptr, int dot_mode = 0);

template <typename T>
void launch_cheb_split(hipStream_t st, const Pair &pr, const TileDims &td, int mode, const T *Sv, const cpx<T> *y,
                       const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta, double c1, double c2,
                       double *partial);

// cluster walk of the Chebyshev step (variant 1): the S blocks in walk order
// (launch_permute_blocks, once per solve) and the fused step over them
template <typename T>
void launch_permute_blocks(hipStream_t st, const Pair &pr, const T *src, T *dst);
template <typename T>
void launch_cheb_cl(hipStream_t st, const Pair &pr, const TileDims &td, int mode, const T *Scl, const cpx<T> *y,
                    const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta, double c1, double c2,
                    double *partial);

// h = H u and s = S u with the split dots of two packed real Lanczos
// processes per column
template <typename T>
void launch_lz_hprod(hipStream_t st, const Pair &pr, const TileDims &td, const T *Hv, const T *Sv, const cpx<T> *u,
                     cpx<T> *h, cpx<T> *su, const int *skip, double *part);

int slab_groups(int nb);
template <typename T>
void launch_spmm_seed_slab(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const T *Hv,
                           const cpx<T> *p, cpx<T> *q, const c128 *z, const int *seed, const int *skip,
                           c128 *partial);
template <typename T>
void launch_spmm_S_slab(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const cpx<T> *d, cpx<T> *w,
                        const int *skip, double *partial);
template <typename T>
void launch_cheb_slab(hipStream_t st, const Pair &pr, const TileDims &td, int mode, const T *Sv, const cpx<T> *y,
                      const cpx<T> *r, cpx<T> *yio, const int *skip, double inv_theta, double c1, double c2,
                      double *partial);

}  // namespace gsc
