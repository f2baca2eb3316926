#pragma once
#include "kernels.h"

namespace gsc {

template <typename T>
void launch_spmm_seed(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const T *Hv,
                      const cpx<T> *p, cpx<T> *q, const c128 *z, const int *seed, const int *skip,
                      c128 *partial);

template <typename T>
void launch_spmm_S(hipStream_t st, const Pair &pr, const TileDims &td, const T *Sv, const cpx<T> *d,
                   cpx<T> *w, const int *skip, double *partial);

}  // namespace gsc
