#pragma once
#include "common.h"

namespace gsc {

void validate_and_upload(Pair &p, int block, int64_t nbrows, const int64_t *rowptr, const int32_t *colidx);
void set_values(Pair &p, const double *H, const double *S, int mem);
double ased_build(Pair &p, const gsc_ased_geom *g, double scale);
void ased_vjp(const Pair &p, const gsc_ased_geom *g, double scale, const double *dH, const double *dS, int mem,
              double *forces);

}  // namespace gsc
