#pragma once
// Charge-self-consistent term (Sec. 2.2, eq. Hap-CSC) on a pair's pattern.
#include "common.h"

namespace gsc {

// Atom pairs coupled by the block pattern (every atom of block row I with
// every atom of block column J, with that block's lattice translation),
// their interaction gamma, and the atom -> orbital map.
struct Csc {
    Ctx *ctx = nullptr;
    int device = 0;             // the context's device (destruction does not read ctx)
    int64_t n_atoms = 0, npairs = 0;
    int B = 0;
    int64_t N = 0, nnzb = 0;
    DevBuf<int32_t> aptr, arow, acol, ablk;   // CSR over atoms; ablk = block of the pair
    DevBuf<double> pos, trans, U, gamma;     // [n_atoms][3], [nnzb][3], [n_atoms], [npairs]
    DevBuf<int32_t> orb_atom, optr, oidx;    // [N]; atom -> orbitals CSR
};

void csc_build(Csc &c, Ctx &ctx, const Pair &p, const gsc_ased_geom &g, const double *U);
// V = gamma dq (device arrays of n_atoms)
void csc_potential(const Csc &c, const double *dq, double *V, hipStream_t st);
// H = H0 + 1/2 S (V_u + V_v) on every stored entry of the pair (device)
void csc_hamiltonian(const Csc &c, Pair &p, const double *H0, const double *V, hipStream_t st);
// dq_out = (sum of q_orb over the atom's orbitals) - Z; f = dq_out - dq_in
void csc_charges(const Csc &c, const double *q_orb, const double *Z, const double *dq_in, double *dq_out, double *f,
                 hipStream_t st);
// max |x| over n entries into *out (device)
void max_abs(int64_t n, const double *x, double *out, hipStream_t st);
// Anderson mixing on the device: dots of the residual differences (out:
// [mh][mh] Gram matrix then [mh] right-hand side) and the combination
//   x_new = x + beta f - sum_i g_i ((x - X_i) + beta (f - F_i))
void anderson_dots(int64_t n, int mh, const double *f, const double *Fh, double *out, hipStream_t st);
void anderson_mix(int64_t n, int mh, double beta, const double *g, const double *x, const double *f,
                  const double *Xh, const double *Fh, double *xnew, hipStream_t st);

// Gradient of a charge-dependent loss (charge_vjp.hip): columns S e_a of
// the listed orbitals (out [R][N] complex) and the accumulation of dL/dH,
// dL/dS on the stored entries from x = G_k e_a and lam = G_k S e_a
// ([K][R][N] complex each).
void launch_s_columns(hipStream_t st, const Pair &p, int R, const int64_t *orbs, c128 *out);
void launch_charge_vjp(hipStream_t st, const Pair &p, int K, int R, const c128 *X, const c128 *Lm, const c128 *z,
                       const double *w, const double *qbar, const int64_t *orbs, double *dH, double *dS);

}  // namespace gsc
