"""Shift grids, quadrature weights and right-hand-side picks."""
from __future__ import annotations

import numpy as np


def shift_grid(e_lo: float, e_hi: float, k: int, eta: float) -> np.ndarray:
    """z_k = E_k + i*eta with E_k uniform on [e_lo, e_hi] (both ends included)."""
    e = np.linspace(e_lo, e_hi, k) if k > 1 else np.array([0.5 * (e_lo + e_hi)])
    return (e + 1j * eta).astype(np.complex128)


def trapezoid_weights(z: np.ndarray) -> np.ndarray:
    """Trapezoid weights in E = Re z for a uniform grid."""
    e = z.real
    k = e.shape[0]
    if k == 1:
        return np.ones(1)
    h = (e[-1] - e[0]) / (k - 1)
    w = np.full(k, h)
    w[0] = w[-1] = 0.5 * h
    return w


def rhs_atoms(rng, n_atoms: int, n_pick: int, block: int) -> np.ndarray:
    """All ``block`` orbitals of ``n_pick`` distinct random atoms (int64)."""
    atoms = rng.choice(n_atoms, size=n_pick, replace=False)
    return (atoms[:, None] * block + np.arange(block)[None, :]).reshape(-1).astype(np.int64)
