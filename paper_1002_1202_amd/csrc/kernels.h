// Device kernels of the generalized shifted COCG solve (Sec. 3.3).
//
// Layouts (one device tile of Rp right-hand sides; Rp is a multiple of 64):
//   seed vectors   v[i*Rp + c]            complex, i < N, c < Rp
//   ring of r'     ring[t][i*Rp + c]      t < m   (r'_n lives in slot n % m)
//   shifted        X[k*ldk + c*N + i]     complex (x^k and p^k, full carry)
//   (k, c) scalars s[k*Rp + c]            FP64
//   column scalars col[c]                 FP64
// A wave of 64 lanes covers 64 consecutive columns; rows are split over the
// grid's y dimension (row groups), remapped so that each XCD works on one
// contiguous range of rows (neighbour reuse stays inside one L2).
#pragma once

#include "common.h"

namespace gsc {

constexpr int kMaxFuse = 16;          // largest m of the fused shift update
constexpr int kHist = 64;             // CG coefficients kept per column for Ritz bounds
constexpr int kFrozenNever = 0x7fffffff;

enum : int { FLAG_BREAKDOWN = 1, FLAG_NOT_SPD = 2, FLAG_NAN = 4, FLAG_INNER = 8 };

// Column (right-hand side) state of one tile, all FP64.
struct ColState {
    c128 *rho, *alpha, *alpha_prev, *beta_prev, *swc, *swcm;
    double *bnorm, *rnorm2, *rr, *rr_stop, *cg_a, *cg_b;
    int *seed, *done, *inner_done, *cg_first, *sw, *applied, *flags, *zres;
    int *inner_count;
    long long *shift_iters;
    int *iters;
    long long *inner_total;   // inner CG steps summed over the solve
    long long *act_hist;      // [max_iter] active (shift, column) pairs per iteration
    long long *col_hist;      // [max_iter] unfinished columns per iteration
    double *cg_ha, *cg_hb;    // [Rp][kHist] CG step sizes and beta of a recorded solve (or null)
    double *wres;             // largest residual over the column's unconverged shifts (-1: none)
};

// (shift, column) state.
struct ShiftState {
    const c128 *z;            // [K]
    c128 *pi, *pi_prev, *pi_next;
    c128 *omega;              // collinear-restart weights (projected carry)
    double *res;              // recursive residual estimate at freeze / exit
    int *last;                // last active step (kFrozenNever while active)
    c128 *ra, *rb, *rc;       // [Rp][K][m] shift-update coefficients (see coef_at)
    // z-derivative carry (null unless requested): d/dz_k of pi, of the
    // restart weight and of the three update coefficients
    c128 *dpi, *dpi_prev, *dpi_next, *domega;
    c128 *rda, *rdb, *rdc;
    int cK = 0, cm = 1;       // shifts and ring depth of the coefficient arrays
};

// Coefficient slot of (shift k, column c, ring slot): the m steps of one
// (column, shift) pair are contiguous, so the fused update fetches all of
// them with one vector load.
__host__ __device__ inline size_t coef_at(const ShiftState &ss, int k, int c, int slot) {
    return (static_cast<size_t>(c) * ss.cK + k) * ss.cm + slot;
}

struct TileDims {
    int N, nb, B, K, R, Rp, m;
    int G;                    // row groups of the vector kernels (multiple of 8)
    int Lr;                   // rows per group (vector kernels)
    int Gs;                   // row groups of the SpMM kernels (multiple of 8); group g, wave w
                              // takes block rows 4g + w + 4 Gs i, i = 0, 1, ...
    bool nt = false;          // streamed vectors of the Chebyshev step bypass L2 retention
    int cb = 0;               // columns per Chebyshev column block (multiple of 64; Rp: one block)
};

// XCD-aware remap of the linear block id: blocks l = x + gx*y are dispatched
// round-robin over the 8 XCDs; give each XCD a contiguous slice of the
// logical (x, y) space.
__device__ inline void xcd_remap(int &cx, int &gy) {
    const int gx = gridDim.x;
    const int total = gx * gridDim.y;
    const int l = blockIdx.x + gx * blockIdx.y;
    const int per = total >> 3;
    const int lp = (l & 7) * per + (l >> 3);
    cx = lp % gx;
    gy = lp / gx;
}

// XCD-aware map for the gathered products: XCD x (= linear id mod 8) owns
// one column chunk (or a set of chunks) and walks its share of the row
// groups in order, so the x rows a chunk needs (its rows plus the
// neighbour halo) are fetched into one L2 instead of into all eight.
__device__ inline void xcd_remap_chunks(int &cx, int &gy) {
    const int gx = gridDim.x, G = gridDim.y;
    const int l = blockIdx.x + gx * blockIdx.y;
    const int x = l & 7, k = l >> 3;
    if (gx <= 8 && (8 % gx) == 0) {
        const int share = 8 / gx;
        cx = x % gx;
        gy = (x / gx) * (G / share) + k;
    } else if ((gx % 8) == 0) {
        cx = x + 8 * (k / G);
        gy = k % G;
    } else {
        xcd_remap(cx, gy);
    }
}

// loads and stores of streamed (read-once / write-once) vector elements;
// NT marks them nontemporal so they do not displace reused lines in L2
template <typename T, bool NT>
__device__ inline T ld_stream(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename T, bool NT>
__device__ inline void st_stream(T v, T *p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename T, bool NT>
__device__ inline cpx<T> ld_cpx(const cpx<T> *p) {
    const T *q = reinterpret_cast<const T *>(p);
    return {ld_stream<T, NT>(q), ld_stream<T, NT>(q + 1)};
}
template <typename T, bool NT>
__device__ inline void st_cpx(cpx<T> v, cpx<T> *p) {
    T *q = reinterpret_cast<T *>(p);
    st_stream<T, NT>(v.re, q);
    st_stream<T, NT>(v.im, q + 1);
}

// Three-term Chebyshev update of one element of S y = r:
//   res = r - S y_k,   y_{k+1} = y_k + c1 (y_k - y_{k-1}) + c2 res.
// own = y_k at this element (taken from the gathered diagonal block), Sx =
// the gathered product.  MODE 0: the first step, whose gathered vector is r
// and y_1 = r / theta, y_0 = 0; MODE 1: y_{k-1} = y_1 = r / theta is formed
// from r; MODE 2: y_{k-1} is read from yprev_src.  Returns y_{k+1}; res2 gets
// |res|^2 and rv the element of r.
template <typename T, int MODE, bool NT>
__device__ inline cpx<T> cheb_next(cpx<T> own, cpx<T> Sx, const cpx<T> *__restrict__ r,
                                   const cpx<T> *__restrict__ yprev_src, size_t e, T inv_theta, T c1, T c2,
                                   double &res2, cpx<T> &rv) {
    cpx<T> yk, yprev, Sy = Sx;
    if constexpr (MODE == 0) {
        rv = own;
        yk = inv_theta * own;
        Sy = inv_theta * Sx;
        yprev = {0, 0};
    } else {
        rv = ld_cpx<T, NT>(r + e);
        yk = own;
        if constexpr (MODE == 1) yprev = inv_theta * rv;
        else yprev = ld_cpx<T, NT>(yprev_src + e);
    }
    const cpx<T> res = rv - Sy;
    res2 = static_cast<double>(res.re) * res.re + static_cast<double>(res.im) * res.im;
    return yk + c1 * (yk - yprev) + c2 * res;
}

// The update above with y_{k+1} written over y_{k-1} (yio).  Returns |res|^2;
// with dacc, also adds y_{k+1} r (unconjugated, FP64) to it.
template <typename T, int MODE, bool NT>
__device__ inline double cheb_update(cpx<T> own, cpx<T> Sx, const cpx<T> *__restrict__ r, cpx<T> *__restrict__ yio,
                                     size_t e, T inv_theta, T c1, T c2, c128 *dacc = nullptr) {
    double res2;
    cpx<T> rv;
    const cpx<T> ynew = cheb_next<T, MODE, NT>(own, Sx, r, yio, e, inv_theta, c1, c2, res2, rv);
    st_cpx<T, NT>(ynew, yio + e);
    if (dacc) *dacc = *dacc + ccast<double>(ynew) * ccast<double>(rv);
    return res2;
}

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// rows handled by wave w of a row group [i0, i1) (waves interleave rows)
__device__ inline int wave_rows(int i0, int i1, int w) {
    const int n = i1 - i0 - w;
    return n > 0 ? (n + kWavesPerBlock - 1) / kWavesPerBlock : 0;
}

}  // namespace gsc
