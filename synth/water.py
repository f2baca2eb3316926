"""Seeded liquid-water box with one 6x6 block per molecule.

Orbitals per molecule (B = 6): O 2s, O 2p x3, H 1s, H 1s.  Oxygens sit on a
random subset of a jittered cubic grid at 1 g/cm^3, molecules are rigid
(O-H 0.9572 A, H-O-H 104.52 deg) with uniformly random orientations.  A
molecule-pair block is stored when the two oxygens are within ``cutoff`` in
the minimum image; the whole 6x6 block is kept.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .system import ASEDParams, TBSystem, csr_from_pairs

EPS_O2S, EPS_O2P, EPS_H1S = -32.3, -14.8, -13.6
R_OH = 0.9572
ANG_HOH = np.deg2rad(104.52)
DENSITY = 0.03343            # molecules per A^3 at 1 g/cm^3


def _random_rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def water_box(n_mol: int = 3000, rng=None, cutoff: float = 6.0, grid: int | None = None,
              jitter: float = 0.3, name: str = "water",
              params: ASEDParams | None = None) -> TBSystem:
    rng = rng if rng is not None else np.random.default_rng(0)
    L = (n_mol / DENSITY) ** (1.0 / 3.0)
    g = grid or int(np.ceil(n_mol ** (1.0 / 3.0)))
    if g ** 3 < n_mol:
        raise ValueError("grid too small")
    h = L / g
    sites = np.stack(np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij"),
                     -1).reshape(-1, 3) * h + h / 2
    pick = np.sort(rng.choice(sites.shape[0], size=n_mol, replace=False))
    o = sites[pick] + rng.uniform(-jitter, jitter, size=(n_mol, 3))
    rot = _random_rotations(rng, n_mol)
    half = ANG_HOH / 2
    h_local = np.array([[np.sin(half), 0.0, np.cos(half)],
                        [-np.sin(half), 0.0, np.cos(half)]]) * R_OH
    hpos = o[:, None, :] + np.einsum("mij,hj->mhi", rot, h_local)
    pos = np.empty((3 * n_mol, 3))
    pos[0::3], pos[1::3], pos[2::3] = o, hpos[:, 0], hpos[:, 1]
    box = np.full(3, L)
    tree = cKDTree(np.mod(o, L), boxsize=box)
    pairs = tree.query_pairs(cutoff, output_type="ndarray")
    pairs = np.sort(pairs, axis=1)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))].astype(np.int64)
    d = o[pairs[:, 1]] - o[pairs[:, 0]]
    trans = -np.round(d / L) * L
    ang = rng.uniform(-1.0, 1.0, size=(pairs.shape[0], 6, 6))
    up = rng.uniform(-1.0, 1.0, size=(n_mol, 6, 6))
    diag = np.triu(up, 1)
    diag = diag + np.transpose(diag, (0, 2, 1))
    rowptr, colidx, transb, angb = csr_from_pairs(n_mol, pairs, trans, ang, diag)
    orb_atom = np.stack([3 * np.arange(n_mol)] * 4 + [3 * np.arange(n_mol) + 1,
                                                      3 * np.arange(n_mol) + 2], 1).reshape(-1)
    eps = np.tile(np.array([EPS_O2S, EPS_O2P, EPS_O2P, EPS_O2P, EPS_H1S, EPS_H1S]), n_mol)
    valence = np.tile(np.array([6.0, 1.0, 1.0]), n_mol)
    return TBSystem(name=name, block=6, positions=pos, orb_atom=orb_atom.astype(np.int64),
                    eps=eps, rowptr=rowptr, colidx=colidx, trans=transb, ang=angb,
                    params=params or ASEDParams(), box=box, valence=valence,
                    meta=dict(n_mol=n_mol, L=L, cutoff=cutoff))
