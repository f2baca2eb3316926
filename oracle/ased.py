"""Dense ASED overlap / Hamiltonian pair (Sec. 2.2, eq. Hap-1) and its
derivative with respect to atomic positions.  FP64, written for clarity.

Model (readings stated in the design notes):
  * on-site: S_{ia,ia} = 1, H_{ia,ia} = eps_{ia} (Sec. 2.2, diagonal rule);
    two orbitals of one atom do not overlap;
  * off-site overlap: S_off = s0 exp(-(r - r0)/lam) * a, with ``a`` the seeded
    angular factor of the stored block and r the distance of the two orbital
    centres (with the block's lattice translation);
  * the off-site part is scaled by c = theta / max_row sum |S_off| so that S is
    diagonally dominant, S = I + c S_off;  c is computed once and is held
    fixed under differentiation;
  * eq. Hap-1 with a constant K: H_{ia,jb} = K (eps_ia + eps_jb)/2 S_{ia,jb}.
"""
from __future__ import annotations

import numpy as np


def _entry_geometry(system):
    """Per stored block: the displacement vector and distance of every entry,
    and a mask of the entries that join two different atoms."""
    B = system.block
    rows = system.block_rows()
    cols = system.colidx.astype(np.int64)
    o1 = rows[:, None] * B + np.arange(B)[None, :]            # (nnzb, B)
    o2 = cols[:, None] * B + np.arange(B)[None, :]
    u = system.orb_atom[o1][:, :, None]                       # atom of the row orbital
    v = system.orb_atom[o2][:, None, :]                       # atom of the column orbital
    d = (system.positions[v] + system.trans[:, None, None, :]
         - system.positions[u])                                # (nnzb, B, B, 3)
    r = np.sqrt(np.sum(d * d, axis=-1))
    same_atom = (u == v) & np.all(system.trans == 0.0, axis=1)[:, None, None]
    return o1, o2, d, r, ~same_atom


def overlap_offsite_blocks(system):
    """Unscaled off-site overlap s(r) * a for every stored entry (nnzb, B, B)."""
    p = system.params
    _, _, _, r, off = _entry_geometry(system)
    s = p.s0 * np.exp(-(r - p.r0) / p.lam) * system.ang
    return np.where(off, s, 0.0)


def scale_constant(system) -> float:
    """c = theta / (largest off-site absolute row sum of the unscaled overlap)."""
    B = system.block
    s = overlap_offsite_blocks(system)
    rows = system.block_rows()
    rowsum = np.zeros(system.n)
    for b in range(system.nnzb):
        rowsum[rows[b] * B:(rows[b] + 1) * B] += np.abs(s[b]).sum(axis=1)
    return float(system.params.theta / rowsum.max())


def pair_blocks(system, c: float | None = None):
    """Stored blocks of S and H, each (nnzb, B, B), plus the scale c used."""
    B = system.block
    if c is None:
        c = scale_constant(system)
    s_off = overlap_offsite_blocks(system)
    o1, o2, _, _, off = _entry_geometry(system)
    diag = (o1[:, :, None] == o2[:, None, :])
    S = np.where(diag, 1.0, c * s_off)
    e1 = system.eps[o1][:, :, None]
    e2 = system.eps[o2][:, None, :]
    H = np.where(diag, e1 * np.ones_like(e2), system.params.kappa * 0.5 * (e1 + e2) * c * s_off)
    del B
    return S, H, c


def dense_pair(system, c: float | None = None):
    """Dense (N, N) S and H in FP64 and the scale c."""
    Sb, Hb, c = pair_blocks(system, c)
    B = system.block
    N = system.n
    S = np.zeros((N, N))
    H = np.zeros((N, N))
    rows = system.block_rows()
    for b in range(system.nnzb):
        I, J = rows[b], int(system.colidx[b])
        S[I * B:(I + 1) * B, J * B:(J + 1) * B] = Sb[b]
        H[I * B:(I + 1) * B, J * B:(J + 1) * B] = Hb[b]
    return S, H, c


def gather_blocks(system, M: np.ndarray) -> np.ndarray:
    """Entries of a dense (N, N) matrix at the stored pattern, (nnzb, B, B)."""
    B = system.block
    rows = system.block_rows()
    out = np.empty((system.nnzb, B, B), dtype=M.dtype)
    for b in range(system.nnzb):
        I, J = rows[b], int(system.colidx[b])
        out[b] = M[I * B:(I + 1) * B, J * B:(J + 1) * B]
    return out


def forces(system, dE_dH: np.ndarray, dE_dS: np.ndarray, c: float) -> np.ndarray:
    """F = -dE/dR through eq. Hap-1 with c, the pattern and the angular
    factors held fixed.  ``dE_dH`` and ``dE_dS`` hold dE/d(entry) for every
    stored entry (nnzb, B, B), each stored entry an independent variable."""
    p = system.params
    o1, o2, d, r, off = _entry_geometry(system)
    e1 = system.eps[o1][:, :, None]
    e2 = system.eps[o2][:, None, :]
    # total derivative of E with respect to the scaled off-site overlap entry
    g = dE_dS + dE_dH * p.kappa * 0.5 * (e1 + e2)
    s = p.s0 * np.exp(-(r - p.r0) / p.lam) * system.ang
    ds_dr = -s / p.lam
    coef = np.where(off, g * c * ds_dr / np.where(off, r, 1.0), 0.0)   # dE/dr / r
    grad_v = coef[..., None] * d           # dE/dR_v  (column-orbital atom)
    u = system.orb_atom[o1][:, :, None] * np.ones_like(system.orb_atom[o2][:, None, :])
    v = system.orb_atom[o2][:, None, :] * np.ones_like(system.orb_atom[o1][:, :, None])
    dEdR = np.zeros_like(system.positions)
    np.add.at(dEdR, v.reshape(-1), grad_v.reshape(-1, 3))
    np.add.at(dEdR, u.reshape(-1), -grad_v.reshape(-1, 3))
    return -dEdR
