"""Green's-function columns by direct factorisation, and the reductions
built on them.  FP64 / complex128 throughout.

Plain definition (Sec. 3.1, eqs. base-2 and GreensFunc, generalised to the
non-orthogonal pair): for every shift z_k and right-hand side b,
    x_k = (z_k S - H)^{-1} b,    G_ij(z_k) = (x_k)_i  for b = e_j.
The matrix z_k S - H is complex symmetric and nonsingular for Im z_k > 0.

Reductions (Sec. 2.2: Mulliken partition of the charge; band energy), spin
factor 2, caller quadrature weights w_k over E_k = Re z_k:
    q_a = -(2/pi) sum_k w_k Im[(S G_k)_aa]
    e_a = -(2/pi) sum_k w_k E_k Im[(S G_k)_aa]
    E_band = sum_a e_a   (sum over all orbitals gives the full band energy)
Gradients of the full band energy with respect to each stored entry:
    dE/dH = -(2/pi) sum_k w_k E_k Im[G_k S G_k]
    dE/dS = -(2/pi) sum_k w_k E_k Im[G_k - z_k G_k S G_k]
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse


def _rhs_matrix(n: int, rhs_idx=None, B_dense=None) -> np.ndarray:
    if B_dense is not None:
        return np.asarray(B_dense, dtype=np.complex128).reshape(n, -1)
    Bm = np.zeros((n, len(rhs_idx)), dtype=np.complex128)
    Bm[np.asarray(rhs_idx), np.arange(len(rhs_idx))] = 1.0
    return Bm


def solve_dense(H: np.ndarray, S: np.ndarray, z, rhs_idx=None, B_dense=None) -> np.ndarray:
    """X[k, r, :] = (z_k S - H)^{-1} b_r by LAPACK LU (zgetrf / zgetrs)."""
    n = H.shape[0]
    Bm = _rhs_matrix(n, rhs_idx, B_dense)
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    X = np.empty((z.shape[0], Bm.shape[1], n), dtype=np.complex128)
    for k, zk in enumerate(z):
        A = zk * S - H
        lu = scipy.linalg.lu_factor(A, check_finite=False)
        X[k] = scipy.linalg.lu_solve(lu, Bm, check_finite=False).T
    return X


def sparse_matrices(system, Sb: np.ndarray, Hb: np.ndarray):
    """CSR S and H assembled from stored blocks (nnzb, B, B)."""
    B = system.block
    rows = system.block_rows()
    r = (rows[:, None, None] * B + np.arange(B)[None, :, None]) * np.ones((1, 1, B), np.int64)
    c = (system.colidx.astype(np.int64)[:, None, None] * B + np.arange(B)[None, None, :]) \
        * np.ones((1, B, 1), np.int64)
    shape = (system.n, system.n)
    S = scipy.sparse.csr_matrix((Sb.reshape(-1), (r.reshape(-1), c.reshape(-1))), shape=shape)
    H = scipy.sparse.csr_matrix((Hb.reshape(-1), (r.reshape(-1), c.reshape(-1))), shape=shape)
    return S, H


def mulliken_band(S, X: np.ndarray, z, w, rhs_idx):
    """q_a, e_a for the orbitals a = rhs_idx from columns X[k, r, :] = G_k e_a,
    and their sum of e_a.  ``S`` may be dense or sparse."""
    z = np.asarray(z, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    rhs_idx = np.asarray(rhs_idx)
    K, R, _ = X.shape
    sg = np.empty((K, R), dtype=np.complex128)          # (S G_k)_aa
    for k in range(K):
        for r in range(R):
            a = rhs_idx[r]
            row = S[a] if not scipy.sparse.issparse(S) else S.getrow(a).toarray()[0]
            sg[k, r] = np.dot(row, X[k, r])
    q = -(2.0 / np.pi) * np.einsum("k,kr->r", w, sg.imag)
    e = -(2.0 / np.pi) * np.einsum("k,kr->r", w * z.real, sg.imag)
    return q, e, float(e.sum())


def band_energy_grad_dense(H, S, z, w):
    """Dense dE/dH and dE/dS (N x N) of the full band energy."""
    z = np.asarray(z, dtype=np.complex128)
    n = H.shape[0]
    gH = np.zeros((n, n))
    gS = np.zeros((n, n))
    for zk, wk in zip(z, w):
        G = np.linalg.inv(zk * S - H)
        GSG = G @ S @ G
        gH += -(2.0 / np.pi) * wk * zk.real * GSG.imag
        gS += -(2.0 / np.pi) * wk * zk.real * (G - zk * GSG).imag
    return gH, gS


def charge_grad_dense(H, S, z, w, orbs, qbar):
    """Dense gradients (N x N) of L = sum_r qbar_r q_{orbs[r]} with respect to
    every entry of H and S, each entry an independent variable.

    From q_a = -(2/pi) sum_k w_k Im[(S G_k)_aa] and dG = G dH G,
    dG = -z G dS G (G = (zS - H)^{-1}, complex symmetric):
        d(S G)_aa / dH_bc = (S G)_ab G_ca,
        d(S G)_aa / dS_bc = delta_ab G_ca - z (S G)_ab G_ca,
    so with Q = diag(qbar on the listed orbitals)
        dL/dH = -(2/pi) sum_k w_k Im[G_k S Q G_k],
        dL/dS = -(2/pi) sum_k w_k Im[Q G_k - z_k G_k S Q G_k].
    (With Q = I and weights w_k E_k this is the band-energy gradient.)"""
    z = np.asarray(z, dtype=np.complex128)
    n = H.shape[0]
    Q = np.zeros((n, n))
    np.add.at(Q, (np.asarray(orbs), np.asarray(orbs)), np.asarray(qbar, dtype=np.float64))
    gH = np.zeros((n, n))
    gS = np.zeros((n, n))
    for zk, wk in zip(z, w):
        G = np.linalg.inv(zk * S - H)
        GSQG = G @ S @ Q @ G
        gH += -(2.0 / np.pi) * wk * GSQG.imag
        gS += -(2.0 / np.pi) * wk * (Q @ G - zk * GSQG).imag
    return gH, gS
