/*
 * gsc.h - generalized shifted COCG on MI355X (gfx950), C ABI.
 *
 * Solves the family of complex-symmetric sparse systems
 *
 *     (z_k S - H) x_k = b,        k = 0 .. nshift-1,
 *
 * for a real symmetric tight-binding Hamiltonian H and a real symmetric
 * positive-definite overlap S that share one block-sparse pattern (the
 * non-orthogonal problem of Sec. 3.1, eqs. base-2 and GreensFunc, written for
 * a general overlap).  One seed COCG process per right-hand side (Sec. 3.3,
 * eqs. CGp:p, CGp:x, CGp:r, S^{-1} r by an inner CG) carries every other shift
 * through the scalar recurrence of eq. Shift:pi and the collinear residual
 * theorem (eq. Collinear); when the seed converges the seed is switched
 * (Sec. 3.3, seed switching) without discarding the Krylov history.
 *
 * Conventions shared by every entry point
 *  - Complex numbers are interleaved (re, im) pairs of double.
 *  - The pattern is block-CSR with B x B blocks (B = 4 or 6): rowptr has
 *    nbrows+1 int64 entries, colidx int32 column-block indices sorted inside
 *    each block row, both triangles stored, every diagonal block present.
 *    Block values are row-major inside the block: val[(b*B + i)*B + j].
 *    N = nbrows * B orbitals.
 *  - gsc_mem says where a pointer lives: GSC_MEM_HOST (pageable host memory)
 *    or GSC_MEM_DEVICE (device memory of the context's device).  Small
 *    inputs (shifts, weights, index lists) are always host memory.
 *  - The caller owns every buffer it passes; the library never frees or
 *    keeps caller pointers beyond the call.  Device work is enqueued on the
 *    context's stream; an entry point returns after its outputs are complete
 *    (it synchronises the stream before returning).
 *  - Every entry point returns a gsc_status.  Negative values are hard
 *    errors (outputs undefined; gsc_last_error() describes the failure).
 *    GSC_NOT_CONVERGED is positive: all outputs are written, together with
 *    per-(shift, rhs) residual estimates and convergence flags in gsc_stats.
 *    Arguments are validated before any device work is launched.
 *  - Results are deterministic: the same inputs and options on the same
 *    device give bitwise-equal outputs, whatever else runs beside them
 *    (every reduction sums its partials in a fixed order; no floating-point
 *    atomics).  Options that change the launch shapes (rhs_tile, cheb_block,
 *    row_groups, fuse_steps) change the summation order and so the last
 *    bits; gsc_solve_batched's scheduling options (batch_streams,
 *    batch_mem_mb, graph_iters) do not (graph_iters only rounds the
 *    reported iteration count up to whole chunks).
 */
#ifndef GSC_H
#define GSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSC_OK = 0,
    GSC_NOT_CONVERGED = 1,
    GSC_E_ARG = -1,          /* invalid argument / malformed pattern        */
    GSC_E_NOMEM = -2,        /* device allocation failed                    */
    GSC_E_DEVICE = -3,       /* HIP runtime error                           */
    GSC_E_BREAKDOWN = -4,    /* COCG breakdown: p^T A p or r'^T r vanished  */
    GSC_E_S_NOT_SPD = -5,    /* inner CG met d^H S d <= 0                    */
    GSC_E_NAN = -6,          /* non-finite value in inputs or iterates      */
    GSC_E_UNSUPPORTED = -7
} gsc_status;

typedef enum { GSC_FP64 = 0, GSC_MIXED = 1, GSC_C64 = 2 } gsc_precision;
typedef enum { GSC_CARRY_FULL = 0, GSC_CARRY_PROJECTED = 1 } gsc_carry;
typedef enum { GSC_MEM_HOST = 0, GSC_MEM_DEVICE = 1 } gsc_mem;

typedef struct gsc_ctx gsc_ctx;
typedef struct gsc_pair gsc_pair;

/* Solver options; gsc_opts_default() fills the defaults given in brackets. */
typedef struct {
    double tol;            /* [1e-10] stop shift k of rhs r once
                              ||r_n|| / (|pi^k_n| ||b||) <= tol (Sec. 3.3,
                              eq. Collinear: the shifted residual is r_n/pi)  */
    int max_iter;          /* [5000] outer iterations                          */
    double inner_tol;      /* [0 = max(1e-2 tol, 1e-15)] relative residual of
                              the inner CG for S r' = r                        */
    int inner_max_iter;    /* [200]                                            */
    int precision;         /* [GSC_FP64] GSC_MIXED: the seed process (products
                              with H and S, seed vectors, dots, recurrences)
                              stays FP64 and the inner S-solve runs complex64
                              Chebyshev rounds (FP32 S and arithmetic) refined
                              by FP64 residuals to the same inner tolerance,
                              so results keep the FP64 accuracy (needs the
                              Chebyshev inner solve; with CG it is FP64).
                              GSC_C64: complex64 vectors and products for the
                              whole seed process, FP64 scalars and dots; its
                              accuracy is limited to about cond(z S - H) times
                              the FP32 epsilon, not by tol                     */
    int carry;             /* [GSC_CARRY_FULL] keep x^k, p^k as full vectors;
                              GSC_CARRY_PROJECTED keeps c^T x^k only and
                              replaces seed switching by a collinear restart   */
    int seed_index;        /* [-1] initial seed shift; -1 = the shift whose
                              real part is nearest the middle of the grid     */
    int fuse_steps;        /* [0 = auto = 16] number m of shift-update steps
                              applied per pass over the shifted vectors (full
                              carry), 1..16                                    */
    int rhs_tile;          /* [0 = auto] right-hand sides per device tile
                              (auto: all that fit; gsc_solve_batched: at most
                              128 per job)                                    */
    int recheck;           /* [0] 1: FP64 true residual of every (k, rhs) into
                              gsc_stats.res_true (full carry only: the
                              projected carry keeps no x_k to check)          */
    int spmm_kernel;       /* [0 = auto = 1] product kernel layout: 1 one block
                              row x 64 rhs per wave (the complex64 steps of
                              GSC_MIXED: 128 rhs per wave, two per lane)      */
    int inner_method;      /* [0 = auto] inner solver for S r' = r: 1 CG (the
                              first solve always runs CG), 2 Chebyshev on the
                              interval of the first CG solve's Ritz values
                              widened by 10 %, with a residual check and extra
                              steps if the check fails; auto = 2 when the
                              interval is positive, else 1                     */
    int graph_iters;       /* [0 = 4] gsc_solve_batched: outer iterations per
                              captured hipGraph launch (between status polls)  */
    int stream_hint;       /* [0 = auto] 1: the Chebyshev step's streamed
                              vectors are loaded and stored with the default
                              cache policy, 2: nontemporal (kept out of L2 so
                              the gathered halo stays resident); auto = 2 for
                              tiles whose automatic column block is one chunk
                              (see cheb_block), else 1                        */
    int cheb_block;        /* [0 = auto] columns per Chebyshev launch block (a
                              multiple of 64, row layout): every step of the
                              inner solve runs on one block of columns at a
                              time; auto sizes the block so that the step's
                              three vectors fit the 256 MB infinity cache
                              (no blocking when the tile already fits; one
                              64-column chunk when not even two chunks fit)   */
    int inner_relax;       /* [0] 1: relaxed inner tolerance (Chebyshev inner
                              solves; gsc_solve_batched captures a job's graph
                              anew when its step count changes): each outer
                              iteration solves S r' = r to inner_tol divided
                              by the largest residual among the shifts still
                              above tol (at most 1e-3, at least inner_tol),
                              so the inner error that reaches every
                              unconverged shift stays at inner_tol relative
                              to ||b||.  0 keeps the fixed inner_tol of the
                              method.                                         */
    int batch_streams;     /* [0 = auto = 8] gsc_solve_batched: jobs (system,
                              rhs tile) iterating concurrently, each on its
                              own stream                                      */
    int batch_mem_mb;      /* [0 = auto] gsc_solve_batched: device memory (MiB)
                              that the workspaces of the jobs iterating at
                              once may hold together.  Jobs start longest
                              first; a job starts when its workspace fits
                              beside those of the live jobs (a job always
                              starts when none is live), and the workspaces
                              of finished jobs are released when a starting
                              job needs their room (else at the end).  auto =
                              80 % of the device memory free at the call.    */
    int row_groups;        /* [0 = auto] workgroup rows of the product and
                              Chebyshev launches (a multiple of 8, at most
                              65528; capped at one block row per wave); auto:
                              one block row per wave while a launch stays
                              within 16384 workgroups, else about 4096
                              workgroups with equal rows per wave             */
    int reserved[1];
} gsc_opts;

/* Statistics.  The three arrays are caller-owned HOST arrays of
 * nshift*nrhs entries laid out [k][r] (any of them may be NULL). */
typedef struct {
    int outer_iters;              /* largest outer iteration count of a tile  */
    long long inner_iters;        /* inner CG steps summed over tiles          */
    int switches;                 /* seed switches summed over rhs            */
    int restarts;                 /* collinear restarts summed over rhs       */
    long long shift_rhs_iters;    /* sum over iterations and rhs of the
                                     number of active shifts                  */
    double seconds;               /* device time of the solve                 */
    double *res_recursive;        /* [k][r] ||r_n|| / (|pi| ||b||) at exit      */
    double *res_true;             /* [k][r] FP64 ||b - A_k x_k|| / ||b||        */
    unsigned char *converged;     /* [k][r] 1 if res_recursive <= tol          */
    double alg_bytes;             /* gsc_solve_batched: algorithmic HBM bytes
                                     of the outer iterations (every vector
                                     element read or written once, each
                                     matrix once per product launch; gathers'
                                     re-reads excluded), 0 elsewhere         */
    double alg_bytes_inner;       /* the inner S-solve's share of alg_bytes   */
} gsc_stats;

/* ASED geometry for gsc_ased_build / gsc_ased_vjp (Sec. 2.2, eq. Hap-1).
 * All arrays are HOST memory.  For stored block b (block row I, column
 * block J) and the entry (a, c) inside it, the orbitals are o1 = I*B + a and
 * o2 = J*B + c; their atoms are u = orb_atom[o1], v = orb_atom[o2] and
 *     d = pos[v] + trans[b] - pos[u],  r = |d|.
 * If u == v and trans[b] == 0 the two orbitals sit on one atom: S = delta,
 * H = delta * eps.  Otherwise S_off = s0 exp(-(r - r0)/lam) ang[b][a][c],
 * S = c S_off and H = kappa (eps[o1] + eps[o2]) / 2 * S, where the scale
 * c = theta / (largest off-site absolute row sum of S_off) keeps S
 * diagonally dominant.  c is computed when scale <= 0, else taken as given
 * (held fixed for derivatives). */
typedef struct {
    int64_t n_atoms;
    const double *pos;        /* [n_atoms][3]            */
    const int32_t *orb_atom;  /* [N]                      */
    const double *eps;        /* [N] on-site levels       */
    const double *trans;      /* [nnzb][3]                */
    const double *ang;        /* [nnzb][B][B]             */
    double s0, r0, lam, kappa, theta;
} gsc_ased_geom;

/* One system of a batched solve (all pointers HOST memory unless noted). */
typedef struct {
    const gsc_pair *pair;
    int nshift;
    const double *z;          /* [nshift] complex                          */
    int nrhs;
    const int64_t *rhs_idx;   /* [nrhs] unit right-hand sides e_j           */
    const double *w;          /* [nshift] quadrature weights or NULL        */
    double *g_diag;           /* out, DEVICE: [nshift][nrhs] complex G_jj   */
    double *q_orb;            /* out, DEVICE: [nrhs] or NULL                */
    double *e_orb;            /* out, DEVICE: [nrhs] or NULL                */
    gsc_stats *stats;         /* optional per-system statistics             */
} gsc_problem;

/* ---- context ------------------------------------------------------------ */
void gsc_opts_default(gsc_opts *opts);
/* Create a context on HIP device `device`; `hip_stream` is a borrowed
 * hipStream_t (NULL = the null stream). */
gsc_status gsc_create(gsc_ctx **out, int device, void *hip_stream);
gsc_status gsc_set_stream(gsc_ctx *ctx, void *hip_stream);
/* Destroys the context and hands the library's cached device blocks and
 * pinned staging buffers back to the runtime. */
void gsc_destroy(gsc_ctx *ctx);
/* The library keeps device blocks of 64 MiB and more after use (per device,
 * up to a third of its memory) and reuses them for later temporaries, so
 * that calls with changing sizes do not pay the kernel driver's clearing of
 * freshly mapped memory; bulk copies of G into host memory go through three pinned
 * 256 MiB staging buffers kept likewise.  This hands every cached block and
 * the staging buffers back to the runtime (for callers that need the memory
 * elsewhere); later calls allocate again. */
gsc_status gsc_release_cache(void);
/* Thread-local description of the last failure ("" if none). */
const char *gsc_last_error(void);
/* Library version string. */
const char *gsc_version(void);

/* ---- the H, S pair (Sec. 3.2: the non-orthogonal basis) ------------------ */
/* Copy the pattern and the FP64 values of H and S to the device.
 * Hval/Sval may be NULL (values set later by gsc_pair_set_values or
 * gsc_ased_build).  GSC_E_ARG for B not in {4, 6}, unsorted or out-of-range
 * column indices, a missing diagonal block or nnzb >= 2^31. */
gsc_status gsc_pair_create(gsc_ctx *ctx, int block, int64_t nbrows,
                           const int64_t *rowptr, const int32_t *colidx,
                           const double *Hval, const double *Sval, int mem,
                           gsc_pair **out);
gsc_status gsc_pair_set_values(gsc_pair *pair, const double *Hval, const double *Sval, int mem);
gsc_status gsc_pair_get_values(const gsc_pair *pair, double *Hval, double *Sval, int mem);
/* Sizes: N, nnzb, block. */
gsc_status gsc_pair_info(const gsc_pair *pair, int64_t *n, int64_t *nnzb, int *block);
/* Frees the pair.  Every other call on a pair needs its context alive; the
 * destruction does not, so pairs and contexts may be destroyed in either
 * order (garbage collectors finalise unreachable objects in any order).
 * The same holds for gsc_csc_destroy. */
void gsc_pair_destroy(gsc_pair *pair);

/* ---- ASED pair (Sec. 2.2, eq. Hap-1) ------------------------------------- */
/* Evaluate S and H on the pair's pattern from the geometry.  scale <= 0:
 * compute c and return it in *scale_out (may be NULL). */
gsc_status gsc_ased_build(gsc_ctx *ctx, const gsc_ased_geom *geom, double scale,
                          gsc_pair *pair, double *scale_out);
/* Forces F = -dE/dpos from dE/dHval and dE/dSval (same block layout as the
 * pair values, each stored entry an independent variable), with the scale c,
 * the pattern and the angular factors held fixed.  dHval/dSval per `mem`;
 * forces: HOST [n_atoms][3]. */
gsc_status gsc_ased_vjp(gsc_ctx *ctx, const gsc_ased_geom *geom, double scale,
                        const gsc_pair *pair, const double *dHval, const double *dSval,
                        int mem, double *forces);

/* ---- products (building blocks of the seed process) ---------------------- */
/* Y = alpha_S * S X - H X for nrhs complex columns stored row-major with the
 * columns interleaved: X[i*nrhs + r] (complex).  alpha_S is one complex
 * scalar per column ([nrhs] complex, HOST).  X, Y per `mem`. */
gsc_status gsc_spmm(gsc_ctx *ctx, const gsc_pair *pair, int nrhs, const double *alpha_S,
                    const double *X, double *Y, int mem);

/* Allocation-free variant of gsc_spmm, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The same product and layout; X and Y are DEVICE
 * memory of the context's device, alpha_S HOST [nrhs] complex.  Its
 * temporaries (per-column shifts, the partial dots of the product kernel,
 * and padded copies of X and Y when nrhs is not a multiple of 64) live in
 * one fixed scratch array of 64 MiB per device, part of the library's code
 * object and held until the process ends; the call performs no device or
 * pinned-host allocation.  GSC_E_ARG, before any device work, when the call
 * needs more than the 64 MiB (with padding about 32 N ceil64(nrhs) bytes).
 * Every call on one device shares that device's scratch, which keeps the
 * last call's contents: calls that overlap on one device (other host
 * threads or other contexts) race and must be serialised by the caller.
 * Synchronises the context's stream before returning. */
gsc_status gsc_spmm_noalloc(gsc_ctx *ctx, const gsc_pair *pair, int nrhs, const double *alpha_S,
                            const double *X, double *Y);

/* ---- the shifted solve (Sec. 3.3) ---------------------------------------- */
/* 1 <= nshift <= 65535 (every entry point that takes shifts).
 * rhs: unit vectors e_{rhs_idx[r]} (rhs_idx HOST [nrhs]) or, if rhs_idx is
 * NULL, dense columns B_dense[r][N] complex (per out_mem); any nrhs (the
 * full carry runs at most 65472 columns per device tile).
 * Outputs (per out_mem; either may be NULL):
 *   G_cols [nshift][nrhs][N] complex   = x_k for rhs r   (full carry only)
 *   G_proj [nshift][nrhs][nproj] complex = (x_k)_{proj_idx[r][m]}
 * proj_idx: HOST [nrhs][nproj] row indices (NULL when nproj == 0). */
gsc_status gsc_solve(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z,
                     int nrhs, const int64_t *rhs_idx, const double *B_dense,
                     const gsc_opts *opts, double *G_cols, int nproj,
                     const int64_t *proj_idx, double *G_proj, int out_mem,
                     gsc_stats *stats);

/* ---- generalised Lanczos + continued fraction (Sec. 3.2) ----------------- */
/* Diagonal Green's-function elements G_jj(z_k), j = rhs_idx[r], by the
 * S-orthonormal three-term recursion of M = S^{-1} H (eqs. 1.13, 1.18)
 * started at S^{-1} e_j, and the continued fraction
 *   G_jj(z) = (S^{-1})_jj / (z - a_0 - b_1^2 / (z - a_1 - b_2^2 / ...)).
 * Each step costs one product with H and one inner solve with S (as in
 * gsc_solve: first solve by CG, then opts->inner_method); no per-shift
 * vectors are kept.  A right-hand side stops when, at a check every
 * check_every steps, its fraction changed by at most tol x max_k |G_jj(z_k)|
 * since the previous check, or when its Krylov space is exhausted; at most
 * m_max steps (check_every = 0: exactly m_max steps).
 * Arguments: rhs_idx HOST [nrhs], 0 <= rhs_idx[r] < N; z HOST [nshift]
 * complex with Im z_k > 0.  Outputs: G_diag [nshift][nrhs] complex (per
 * out_mem); coef_a, coef_b HOST [nrhs][m_max] (may be NULL): a_n and b_n of
 * each right-hand side (b_0 = 0; entries past its step count are 0); steps
 * HOST [nrhs] (may be NULL).  Uses opts->precision, inner_tol,
 * inner_max_iter, inner_method, rhs_tile (right-hand sides per tile).
 * Returns GSC_NOT_CONVERGED when some right-hand side used all m_max steps
 * with checks enabled (outputs are still written), GSC_E_ARG for invalid
 * arguments. */
gsc_status gsc_lanczos_green(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, int nrhs,
                             const int64_t *rhs_idx, int m_max, double tol, int check_every,
                             const gsc_opts *opts, double *G_diag, double *coef_a, double *coef_b,
                             int *steps, int out_mem, gsc_stats *stats);

/* Gradient of a loss of the Mulliken charges, L = sum_r qbar[r] q_{orb_idx[r]}
 * (Sec. 2.2), on every stored entry of H and S (each an independent
 * variable), accumulated into dHval, dSval ([nnzb][B][B] per mem):
 *   dL/dH = -(2/pi) sum_k w_k Im[G_k S Q G_k],
 *   dL/dS = -(2/pi) sum_k w_k Im[Q G_k - z_k G_k S Q G_k],   Q = diag(qbar).
 * For every listed orbital a the shifted solver runs twice (full carry):
 * x = G_k e_a and lam = G_k S e_a, combined on the pattern.  Memory
 * 2 nshift N x (orbitals per tile) complex; for small and medium systems.
 * z, w, orb_idx, qbar HOST.  GSC_NOT_CONVERGED if a solve did not converge
 * (gradients still written). */
gsc_status gsc_charge_vjp(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z, const double *w,
                          int norb, const int64_t *orb_idx, const double *qbar, const gsc_opts *opts,
                          double *dHval, double *dSval, int mem, gsc_stats *stats);

/* ---- charge self-consistency (Sec. 2.2, eq. Hap-CSC) --------------------- */
/*   H^CSC_{ia,jb} = 1/2 S_{ia,jb} sum_k (gamma_ik + gamma_jk) dq_k
 *                 = 1/2 S_{ia,jb} (V_i + V_j),   V = gamma dq,
 * dq_k = Mulliken electron count of atom k minus its valence.  gamma (the
 * paper does not give it): on the atom pairs the pair's block pattern
 * couples (every atom of block row I with every atom of block column J,
 * displaced by that block's translation), gamma_ii = U_i for an atom with
 * itself, else e^2 / sqrt(r^2 + a^2) with a = e^2 (1/U_i + 1/U_k) / 2 and
 * e^2 = 14.399645 eV A (Klopman-Ohno). */
typedef struct gsc_csc gsc_csc;
/* geom: positions, orb_atom and block translations as for gsc_ased_build
 * (HOST); hubbard_u HOST [n_atoms], > 0 (eV).  The handle keeps device
 * copies and gamma; it belongs to the pair's context and device. */
gsc_status gsc_csc_create(gsc_ctx *ctx, const gsc_pair *pair, const gsc_ased_geom *geom, const double *hubbard_u,
                          gsc_csc **out);
void gsc_csc_destroy(gsc_csc *csc);
/* V = gamma dq; dq, V [n_atoms] per mem. */
gsc_status gsc_csc_potential(gsc_csc *csc, const double *dq, double *V, int mem);
/* The pair's H values become H0 + H^CSC(dq) on every stored entry (S of
 * the pair); H0 [nnzb][B][B] and dq [n_atoms] per mem. */
gsc_status gsc_csc_hamiltonian(gsc_csc *csc, gsc_pair *pair, const double *H0, const double *dq, int mem);
/* Self-consistency loop.  H0 is the pair's H at entry.  Each iteration sets
 * H = H0 + H^CSC(dq_in), computes the Mulliken charges of every orbital with
 * the shifts z and weights w (HOST [nshift]) by the projected shifted solve,
 * dq_out = atom sums - valence (HOST [n_atoms]); it stops when
 * max |dq_out - dq_in| <= tol, else takes the next dq_in by Anderson mixing
 * of the last `history` residuals with step beta (history 0: linear mixing
 * dq_in += beta (dq_out - dq_in)).  dq: HOST [n_atoms], the starting charges
 * on entry and the last dq_in on exit; q_orb HOST [N] (the last charges) and
 * e_band HOST may be NULL.  On exit the pair holds H0 + H^CSC(dq).
 * GSC_NOT_CONVERGED after max_iter iterations (outputs written). */
typedef struct {
    double beta;          /* [0.2]  mixing step                            */
    int history;          /* [4]    Anderson history (0 = linear mixing)    */
    double tol;           /* [1e-8] max |dq_out - dq_in| to stop            */
    int max_iter;         /* [100]                                          */
    int neutral;          /* [0] 1: charge neutrality sets the Fermi level
                             each iteration: E_F solves
                             -(2/pi) sum_k w_k(E_F) sum_a Im (S G_k)_aa
                               = sum of the valences
                             (bisection), with w_k(E_F) the trapezoid
                             weights over Re z_k truncated at E_F (the
                             integrand linear between samples); w is then
                             not used (may be NULL), Re z must increase
                             and the grid must reach past E_F             */
} gsc_scc_opts;
void gsc_scc_opts_default(gsc_scc_opts *o);
/* e_fermi: HOST, may be NULL; the last E_F in neutral mode (else the top
 * of the grid, Re z_{nshift-1}).  GSC_E_ARG in neutral mode when Re z is
 * not increasing or the grid holds fewer electrons than the valences. */
gsc_status gsc_scc(gsc_ctx *ctx, gsc_csc *csc, gsc_pair *pair, int nshift, const double *z, const double *w,
                   const double *valence, const gsc_scc_opts *sopts, const gsc_opts *opts, double *dq, double *q_orb,
                   double *e_band, int *iters, double *residual, double *e_fermi);

/* Mulliken charge and band energy per orbital a = orb_idx[r] (Sec. 2.2),
 * spin 2, quadrature weights w[k] (HOST) over E_k = Re z_k:
 *   q_a = -(2/pi) sum_k w_k Im[(S G_k)_aa],
 *   e_a = -(2/pi) sum_k w_k E_k Im[(S G_k)_aa],
 *   *e_band = sum_r e_{orb_idx[r]}  (the band energy when every orbital is
 *   listed).  q_orb, e_orb: [norb] per out_mem; e_band: HOST. */
gsc_status gsc_mulliken_band(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z,
                             const double *w, int norb, const int64_t *orb_idx,
                             const gsc_opts *opts, double *q_orb, double *e_orb,
                             double *e_band, int out_mem, gsc_stats *stats);

/* Backward of the band energy E = sum_a e_a over all orbitals (Sec. 2.2 with
 * the gradient of the Green's function, dG = G dH G, dG = -z G dS G):
 *   dH += grad_E * dE/dH_bc = -(2/pi) sum_k w_k E_k Im[(G_k S G_k)_bc]
 *   dS += grad_E * dE/dS_bc = -(2/pi) sum_k w_k E_k Im[(G_k - z_k G_k S G_k)_bc]
 * on the stored entries (block layout of the pair values, per `mem`).
 * Column c of both gradients comes from the solve with right-hand side e_c
 * alone: G S G e_c = -dx(z)/dz is carried alongside the shifted iterates, so
 * the backward reuses the same shifted solver.  The call covers the columns
 * c = orb_idx[0 .. norb-1] (HOST, distinct, in range; orb_idx == NULL with
 * norb == N: every orbital): it adds those columns of the full gradient and
 * writes *e_band (HOST, may be NULL) = sum over the listed c of e_c.  Calls
 * over a partition of the orbitals therefore add up to the gradient and the
 * value of the full band energy (a caller can split a large system into
 * slices).  GSC_E_ARG for a repeated or out-of-range orbital. */
gsc_status gsc_band_energy_vjp(gsc_ctx *ctx, const gsc_pair *pair, int nshift, const double *z,
                               const double *w, int norb, const int64_t *orb_idx, double grad_E,
                               const gsc_opts *opts, double *dHval, double *dSval, double *e_band,
                               int mem, gsc_stats *stats);

/* ---- kernel timing ------------------------------------------------------- */
/* Live per-kernel timing with HIP events recorded on the context's stream
 * around every launch of the named kernels (for roofline reporting).
 * gsc_profile_enable(ctx, 1) resets the counters and turns timing on.
 * gsc_profile_read returns, for one kernel name ("spmm_seed", "spmm_S",
 * "shift_update", "cg_update", "cg_dir", "update_r", "rho_dot", "p_update",
 * "ctrl", "post", "proj_update", "cheb_step", "ring_transpose", the mixed
 * inner solve's "cheb_mx" (complex64 steps) and "mx_resid" (FP64 residuals),
 * and for the generalised Lanczos process "lz_hprod", "lz_update",
 * "lz_scale"), the summed
 * device milliseconds, the number of launches and the summed algorithmic
 * bytes those launches must move (the method's own reads and writes, no re-reads).  GSC_E_ARG for an
 * unknown name. */
gsc_status gsc_profile_enable(gsc_ctx *ctx, int on);
/* Restrict the event timing to one kernel name (NULL: time every kernel);
 * byte counting continues for all kernels.  Event pairs cost a few
 * microseconds each, so timing one kernel keeps the run undisturbed. */
gsc_status gsc_profile_select(gsc_ctx *ctx, const char *kernel);
gsc_status gsc_profile_read(gsc_ctx *ctx, const char *kernel, double *total_ms, long long *launches,
                            double *bytes);

/* Many independent systems solved together (each system's shifts, rhs and
 * outputs as in gsc_problem).  Projected carry: G_jj for every unit rhs e_j
 * and, when w is given, the Mulliken charge and band-energy contribution of
 * orbital j.  Every (system, rhs tile) is one job; after its set-up each job
 * iterates as a captured hipGraph of opts->graph_iters outer iterations,
 * jobs run concurrently on several streams and a host scheduler polls their
 * completion events (longest jobs first).  Returns GSC_NOT_CONVERGED if any
 * system did not converge (outputs written), a negative status on error. */
gsc_status gsc_solve_batched(gsc_ctx *ctx, int nsys, const gsc_problem *problems,
                             const gsc_opts *opts);

#ifdef __cplusplus
}
#endif
#endif /* GSC_H */
