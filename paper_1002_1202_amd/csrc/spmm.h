#pragma once
#include "kernels.h"

namespace gsc {

// row groups of the product kernels (one block row per wave and step)
void set_spmm_geometry(TileDims &td, const Pair &pr);

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

// mixed inner solve: one complex64 Chebyshev step (FP32 S, FP32 arithmetic)
// for S y = f, mode as launch_cheb_step; fin 0 stores y_{k+1} over y_{k-1},
// fin 1 writes Y = y_{k+1}, fin 2 adds Y += y_{k+1} (Y complex128), with dot
// also the partials of Y^T r into dpart.  launch_mx_resid: f = r - S Y (FP64)
// in complex64 and the partials of ||f||^2.
void launch_cheb_mx(hipStream_t st, const Pair &pr, const TileDims &td, int mode, int fin, bool dot, int col0,
                    int ncols, const float *Sv, const c64 *y, const c64 *f, c64 *yio, c128 *Y, const c128 *r,
                    const int *skip, double inv_theta, double c1, double c2, double *partial, c128 *dpart,
                    int dot_active_only);
void launch_mx_resid(hipStream_t st, const Pair &pr, const TileDims &td, int col0, int ncols, const double *Sv,
                     const c128 *Y, const c128 *r, c64 *f, const int *skip, double *partial);

// h = H u and s = S u with the split dots of two packed real Lanczos
// processes per column
template <typename T>
void launch_lz_hprod(hipStream_t st, const Pair &pr, const TileDims &td, const T *Hv, const T *Sv, const cpx<T> *u,
                     cpx<T> *h, cpx<T> *su, const int *skip, double *part);

}  // namespace gsc
