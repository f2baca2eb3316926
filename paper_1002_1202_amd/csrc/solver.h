#pragma once
#include "kernels.h"

namespace gsc {

struct Status {
    int active_cols;       // columns with at least one unconverged shift
    int inner_pending;     // columns whose inner S-solve has not converged
    int switched;          // columns that switched seed (or restarted) this iteration
    int flags;             // OR of FLAG_* over columns
    double worst_res;      // largest shifted residual still above tol, over columns (-1: none)
    long long col_iters;   // outer iterations summed over the columns so far
};

// Projections carried by the projected mode: M unit vectors c_m = e_i per
// column (idx[c*M + m] = i, for G_ij), optionally followed by c = S e_a with
// a the column's unit right-hand side (for (S G)_aa, the Mulliken charge).
struct ProjSpec {
    int M = 0;                          // unit projections e_i per column
    bool srow = false;                  // also carry c = S e_a, a = rhs[c] (last slot)
    std::vector<int32_t> idx;           // [R][M]
};

struct SolveRequest {
    const Pair *pair = nullptr;
    int K = 0;
    const double *z = nullptr;          // host, 2K
    int R = 0;
    const int64_t *rhs_idx = nullptr;   // host
    const double *B_dense = nullptr;    // [R][N] complex, per out_mem
    gsc_opts opts{};
    // full carry outputs
    double *G_cols = nullptr;           // [K][R][N] complex
    int nproj = 0;
    const int64_t *proj_idx = nullptr;  // host [R][nproj]
    double *G_proj = nullptr;           // [K][R][nproj] complex
    int out_mem = GSC_MEM_HOST;
    // projected carry: projection spec and output [K][R][M] complex (device)
    const ProjSpec *proj = nullptr;
    c128 *proj_out = nullptr;           // device [K][R][M]
    // (S G)_aa for unit rhs: device [K][R] complex (full carry Mulliken path)
    c128 *sg_diag = nullptr;
    // backward: z-derivative carry with quadrature-weighted accumulation,
    // wE = w_k Re z_k (device [K]); acc device [R][M][3] (M = proj M + srow)
    bool vjp = false;
    const double *wE = nullptr;
    c128 *vjp_acc = nullptr;
    gsc_stats *stats = nullptr;
};

gsc_status run_solve(Ctx &ctx, SolveRequest &req);

// Generalised Lanczos + continued fraction for G_jj (unit right-hand sides).
struct LanczosRequest {
    const Pair *pair = nullptr;
    int K = 0;
    const double *z = nullptr;          // host, 2K
    int P = 0;                          // number of right-hand sides e_j
    const int64_t *rhs_idx = nullptr;   // host [P]
    int m_max = 0;
    double tol = 0.0;
    int check_every = 0;
    gsc_opts opts{};
    double *G_diag = nullptr;           // [K][P] complex, per out_mem
    double *coef_a = nullptr;           // host [P][m_max] or null
    double *coef_b = nullptr;           // host [P][m_max] or null
    int *steps = nullptr;               // host [P] or null
    int out_mem = GSC_MEM_HOST;
    gsc_stats *stats = nullptr;
};
gsc_status run_lanczos(Ctx &ctx, LanczosRequest &req);
// Many projected-carry solves at once: one job per (system, rhs tile), each
// iterating as a captured hipGraph of `graph_iters` outer iterations on one
// of up to `max_streams` streams; iters[s] receives the iterations run.
gsc_status run_batched(Ctx &ctx, std::vector<SolveRequest> &reqs, int graph_iters, int max_streams,
                       std::vector<int> &iters);

}  // namespace gsc
