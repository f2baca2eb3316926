"""Container for one synthetic tight-binding geometry.

A ``TBSystem`` carries only *inputs*: atomic positions, the frozen block
sparsity pattern, the periodic image translation of every stored block, the
seeded random orbital angular factors and the on-site levels.  It holds none
of the method's arithmetic: turning these inputs into the overlap S and the
ASED Hamiltonian H (Sec. 2.2, eq. Hap-1) is done separately by the oracle and
by the HIP builder.

Layout conventions shared by every consumer:

* orbitals are numbered ``block * B + slot``; block ``I`` is an atom (Si, B=4:
  s, px, py, pz) or a whole molecule (water, B=6: O 2s, O 2p x3, H 1s, H 1s);
* ``orb_atom[o]`` is the atom that carries orbital ``o``;
* the pattern is block-CSR: ``rowptr`` (int64, nb+1), ``colidx`` (int32, sorted
  per block row, both triangles stored, the diagonal block always present);
* ``trans[b]`` (float64, 3) is the lattice translation added to the position of
  the column block's atoms for stored block ``b``; ``trans`` of the mirrored
  block is the negation;
* ``ang[b]`` (float64, B x B) is the random angular factor of stored block
  ``b``; the mirrored block stores the transpose, so the assembled matrices are
  exactly symmetric.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class ASEDParams:
    """Parameters of the distance law and of eq. Hap-1.

    s(r) = s0 * exp(-(r - r0) / lam) multiplies the angular factor; the whole
    off-site overlap is then scaled by one constant so that the largest
    off-site absolute row sum equals ``theta`` (S stays diagonally dominant).
    ``kappa`` is the constant K of eq. Hap-1.
    """

    s0: float = 0.3
    r0: float = 2.35
    lam: float = 0.8
    kappa: float = 1.75
    theta: float = 0.5


@dataclass
class TBSystem:
    name: str
    block: int                       # B
    positions: np.ndarray            # (n_atoms, 3) float64, Angstrom
    orb_atom: np.ndarray             # (N,) int64
    eps: np.ndarray                  # (N,) float64, eV
    rowptr: np.ndarray               # (nb+1,) int64
    colidx: np.ndarray               # (nnzb,) int32
    trans: np.ndarray                # (nnzb, 3) float64
    ang: np.ndarray                  # (nnzb, B, B) float64
    params: ASEDParams = field(default_factory=ASEDParams)
    box: np.ndarray | None = None    # (3,) periodic lengths (inf = open)
    valence: np.ndarray | None = None  # (n_atoms,) core charge Z per atom
    meta: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def n(self) -> int:
        return self.nb * self.block

    @property
    def nnzb(self) -> int:
        return int(self.colidx.shape[0])

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    def block_rows(self) -> np.ndarray:
        """Block-row index of every stored block (int64, nnzb)."""
        return np.repeat(np.arange(self.nb, dtype=np.int64), np.diff(self.rowptr))

    def mirror(self) -> np.ndarray:
        """Index of the stored block (J, I) for every stored block (I, J)."""
        rows = self.block_rows()
        key = rows * self.nb + self.colidx.astype(np.int64)
        mkey = self.colidx.astype(np.int64) * self.nb + rows
        order = np.argsort(key)
        pos = np.searchsorted(key[order], mkey)
        return order[pos]


def csr_from_pairs(nb: int, pairs: np.ndarray, pair_trans: np.ndarray,
                   pair_ang: np.ndarray, diag_ang: np.ndarray):
    """Assemble the symmetric block pattern from unordered pairs.

    ``pairs`` (P, 2) with i < j, ``pair_trans`` (P, 3) = translation for the
    (i, j) block, ``pair_ang`` (P, B, B) the angular block for (i, j).  The
    diagonal block of every row is added with zero translation and the angular
    block ``diag_ang[i]``.  Returns rowptr, colidx, trans, ang sorted by
    (row, col).
    """
    B = pair_ang.shape[1] if pair_ang.size else diag_ang.shape[1]
    i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    rows = np.concatenate([i, j, np.arange(nb, dtype=np.int64)])
    cols = np.concatenate([j, i, np.arange(nb, dtype=np.int64)])
    trans = np.concatenate([pair_trans, -pair_trans, np.zeros((nb, 3))])
    ang = np.concatenate([pair_ang, np.transpose(pair_ang, (0, 2, 1)), diag_ang])
    order = np.lexsort((cols, rows))
    rows, cols, trans, ang = rows[order], cols[order], trans[order], ang[order]
    counts = np.bincount(rows, minlength=nb)
    rowptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    # the pattern must not hold one block twice (two images of one pair)
    key = rows * nb + cols
    if np.any(np.diff(key) == 0):
        raise ValueError("duplicate block in pattern: cell too small for the cutoff")
    return rowptr, cols.astype(np.int32), np.ascontiguousarray(trans), \
        np.ascontiguousarray(ang.reshape(-1, B, B))
