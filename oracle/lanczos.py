"""Generalised Lanczos process and the continued fraction of G_jj(z).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64, plain code written
from Sec. 3.2 (eqs. 1.13 and 1.18).

For the non-orthogonal pair the section works with the operator
M = S^{-1} H, which is self-adjoint in the S-product (u, w) = u^T S w (real
vectors here: S, H and e_j are real).  The three-term recursion

    M u^n = a_n u^n + b_{n+1} u^{n+1} + b_n u^{n-1},   b_0 = 0, b_n > 0,

with S-orthonormal u^n tridiagonalises M on the Krylov space of the start
vector.  Reading used here (the section does not spell out the start vector
or the read-out): for the diagonal element G_jj(z) of G = (zS - H)^{-1},

    G = (z - M)^{-1} S^{-1},  so  G_jj = e_j^T (z - M)^{-1} v,  v = S^{-1} e_j,
    and since e_j = S v:       G_jj = (v, (z - M)^{-1} v),

the process starts from u^0 = v / ||v||_S with ||v||_S^2 = v^T S v = v_j, and

    G_jj(z) = v_j [(z - T)^{-1}]_00
            = v_j / (z - a_0 - b_1^2 / (z - a_1 - b_2^2 / (z - a_2 - ...)))

truncated after m steps.  Each step needs one product with H and one solve
with S (done exactly here, by a sparse LU factorisation of S).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


class _SSolver:
    """Exact solves with S (dense or sparse), factorised once."""

    def __init__(self, S):
        if scipy.sparse.issparse(S):
            self._lu = scipy.sparse.linalg.splu(scipy.sparse.csc_matrix(S))
            self.solve = self._lu.solve
        else:
            self._cf = scipy.linalg.cho_factor(np.asarray(S, dtype=np.float64))
            self.solve = lambda b: scipy.linalg.cho_solve(self._cf, b)


def lanczos(H, S, j: int, m: int, return_basis: bool = False):
    """m steps of the generalised Lanczos process started at S^{-1} e_j.

    Returns (a[0..m-1], b[0..m-1] with b[0] = 0 and b[n] the coupling of steps
    n-1 and n, v_j = ||S^{-1} e_j||_S^2) and, if asked, the basis U (n x m).
    The process stops early (shorter arrays) if some b_{n+1} vanishes: the
    Krylov space is then exhausted and the fraction is exact."""
    n = H.shape[0]
    Ss = _SSolver(S)
    e = np.zeros(n)
    e[j] = 1.0
    v = Ss.solve(e)
    vj = float(v[j])                      # v^T S v = v^T e_j
    u = v / np.sqrt(vj)
    u_prev = np.zeros(n)
    b_n = 0.0
    a, b, U = [], [0.0], []
    for step in range(m):
        U.append(u)
        Hu = H @ u
        a_n = float(u @ Hu)               # (u, M u) = u^T S S^{-1} H u
        w = Ss.solve(Hu) - a_n * u - b_n * u_prev
        a.append(a_n)
        if step == m - 1:
            break
        b_next = float(np.sqrt(max(w @ (S @ w), 0.0)))
        if b_next <= 1e-14 * max(1.0, abs(a_n)):
            break
        u_prev, u, b_n = u, w / b_next, b_next
        b.append(b_next)
    a = np.array(a)
    b = np.array(b[:len(a)])
    if return_basis:
        return a, b, vj, np.stack(U, axis=1)
    return a, b, vj


def continued_fraction(z, a, b, vj):
    """v_j [(z - T)^{-1}]_00 for the tridiagonal T(a, b), evaluated from the
    bottom of the fraction upwards, for every shift in z."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    t = z - a[-1]
    for n in range(len(a) - 2, -1, -1):
        t = z - a[n] - b[n + 1] ** 2 / t
    return vj / t


def green_diag(H, S, z, rhs, m: int):
    """G_jj(z_k) for every shift and every j in rhs, m Lanczos steps each.
    Returns an array [K][len(rhs)]."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    out = np.empty((z.shape[0], len(rhs)), dtype=np.complex128)
    for c, j in enumerate(rhs):
        a, b, vj = lanczos(H, S, int(j), m)
        out[:, c] = continued_fraction(z, a, b, vj)
    return out


def tridiagonal(a, b):
    """The m x m matrix T of the recursion (diagonal a, off-diagonal b[1:])."""
    T = np.diag(np.asarray(a, dtype=np.float64))
    off = np.asarray(b[1:len(a)], dtype=np.float64)
    return T + np.diag(off, 1) + np.diag(off, -1)
