"""Seeded silicon geometries with an sp3 basis (B = 4 orbitals per atom).

Every builder draws from one ``numpy.random.Generator`` in a fixed order:
positions -> displacements / strain / vacancies -> pattern -> angular blocks,
so a given seed always gives the same system.  The neighbour pattern is taken
from the *ideal* lattice (first and second shells of diamond, 4 + 12
neighbours) so that it stays fixed while atoms move; distances for the
overlap law are always taken from the actual positions.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .system import ASEDParams, TBSystem, csr_from_pairs

A_SI = 5.431                     # diamond lattice constant, Angstrom
EPS_S, EPS_P = -13.6, -6.5       # on-site levels, eV
SHELL2_CUT = 4.0                 # between 2nd (3.840) and 3rd (4.503) shell

_BASIS = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                   [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])


def diamond_lattice(nx: int, ny: int, nz: int, a: float = A_SI) -> np.ndarray:
    """Ideal diamond positions of nx*ny*nz conventional cells (8 atoms each)."""
    cells = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                                 indexing="ij"), -1).reshape(-1, 3)
    pos = (cells[:, None, :] + _BASIS[None, :, :]).reshape(-1, 3) * a
    return pos.astype(np.float64)


def neighbour_pairs(ideal: np.ndarray, box: np.ndarray, periodic: np.ndarray,
                    cutoff: float):
    """Unordered pairs (i < j) closer than ``cutoff`` in the minimum image.

    Returns the pairs and, per pair, the lattice translation to add to atom j
    so that ``pos[j] + T - pos[i]`` is the short bond vector.
    """
    lo = ideal.min(0)
    shifted = ideal - lo
    span = shifted.max(0)
    bs = np.where(periodic, box, span + 4 * cutoff + 1.0)
    shifted = np.mod(shifted, bs)
    tree = cKDTree(shifted, boxsize=bs)
    pairs = tree.query_pairs(cutoff, output_type="ndarray")
    pairs = np.sort(pairs, axis=1)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
    d = ideal[pairs[:, 1]] - ideal[pairs[:, 0]]
    img = np.where(periodic, np.round(d / np.where(periodic, box, 1.0)), 0.0)
    trans = -img * np.where(periodic, box, 0.0)
    return pairs.astype(np.int64), trans


def _si_orbitals(n_atoms: int):
    orb_atom = np.repeat(np.arange(n_atoms, dtype=np.int64), 4)
    eps = np.tile(np.array([EPS_S, EPS_P, EPS_P, EPS_P]), n_atoms)
    return orb_atom, eps


def _assemble(name, pos, box, periodic, pairs, trans_ideal_img, rng, meta,
              params=None):
    """Draw the angular blocks in canonical pair order and build the system."""
    n_atoms = pos.shape[0]
    ang = rng.uniform(-1.0, 1.0, size=(pairs.shape[0], 4, 4))
    diag = np.zeros((n_atoms, 4, 4))
    rowptr, colidx, trans, angb = csr_from_pairs(n_atoms, pairs, trans_ideal_img, ang, diag)
    orb_atom, eps = _si_orbitals(n_atoms)
    return TBSystem(name=name, block=4, positions=pos, orb_atom=orb_atom, eps=eps,
                    rowptr=rowptr, colidx=colidx, trans=trans, ang=angb,
                    params=params or ASEDParams(),
                    box=np.where(periodic, box, np.inf),
                    valence=np.full(n_atoms, 4.0), meta=meta)


def si_bulk(cells=(2, 2, 2), rng=None, sigma: float = 0.0, strain: float = 0.0,
            strain_axis: int | None = None, vacancy_frac: float = 0.0,
            name: str = "si-bulk", params: ASEDParams | None = None) -> TBSystem:
    """Periodic diamond Si with optional Gaussian displacements, uniaxial
    tensile strain and random vacancies; pattern = ideal 1st + 2nd shells."""
    rng = rng if rng is not None else np.random.default_rng(0)
    nx, ny, nz = cells
    ideal = diamond_lattice(nx, ny, nz)
    box = np.array([nx, ny, nz], dtype=np.float64) * A_SI
    periodic = np.array([True, True, True])
    pos = ideal.copy()
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    scale = np.ones(3)
    if strain > 0:
        ax = int(rng.integers(0, 3)) if strain_axis is None else int(strain_axis)
        scale[ax] = 1.0 + strain
    pos = pos * scale
    if vacancy_frac > 0:
        n_vac = int(round(vacancy_frac * ideal.shape[0]))
        drop = rng.choice(ideal.shape[0], size=n_vac, replace=False)
        keep = np.setdiff1d(np.arange(ideal.shape[0]), drop)
        ideal, pos = ideal[keep], pos[keep]
    pairs, trans = neighbour_pairs(ideal, box, periodic, SHELL2_CUT)
    trans = trans * scale
    meta = dict(cells=tuple(cells), sigma=sigma, strain=strain, vacancy_frac=vacancy_frac)
    return _assemble(name, pos, box * scale, periodic, pairs, trans, rng, meta, params)


def si_slab_001(cells=(8, 8, 16), rng=None, dimer_shift: float = 0.7,
                name: str = "si-slab001", params: ASEDParams | None = None) -> TBSystem:
    """(001) slab, periodic in x and y, open in z (vacuum), whose top layer is
    paired into disjoint [110] neighbours that move ``dimer_shift`` toward
    each other.  The pattern is the topological one of the ideal slab."""
    rng = rng if rng is not None else np.random.default_rng(0)
    nx, ny, nz = cells
    ideal = diamond_lattice(nx, ny, nz)
    box = np.array([nx * A_SI, ny * A_SI, nz * A_SI + 20.0])
    periodic = np.array([True, True, False])
    pos = ideal.copy()
    ztop = ideal[:, 2].max()
    top = np.flatnonzero(np.abs(ideal[:, 2] - ztop) < 1e-6)
    # coordinates along [110] (u) and [1-10] (v) in units of a/2
    u = np.round((ideal[top, 0] + ideal[top, 1]) / (A_SI / 2)).astype(np.int64)
    v = np.round((ideal[top, 0] - ideal[top, 1]) / (A_SI / 2)).astype(np.int64)
    period = 2 * nx      # line length along [110] in steps (nx == ny assumed)
    lines = {}
    for k, (uu, vv) in enumerate(zip(u, v)):
        lines.setdefault(int(vv) % period, []).append((int(uu) % period, top[k]))
    partner = {}
    for members in lines.values():
        members.sort()
        for m in range(0, len(members) - 1, 2):
            a_, b_ = members[m][1], members[m + 1][1]
            partner[a_] = b_
            partner[b_] = a_
    L = box[:2]
    for a_, b_ in partner.items():
        d = ideal[b_, :2] - ideal[a_, :2]
        d = d - L * np.round(d / L)
        pos[a_, :2] += dimer_shift * d / np.linalg.norm(d)
    pairs, trans = neighbour_pairs(ideal, box, periodic, SHELL2_CUT)
    meta = dict(cells=tuple(cells), dimer_shift=dimer_shift, n_dimer_atoms=len(partner))
    return _assemble(name, pos, box, periodic, pairs, trans, rng, meta, params)


def si_crack_111(cells=(4, 4, 4), rng=None, opening: float = 1.5, cutoff: float = 4.2,
                 name: str = "si-crack111", params: ASEDParams | None = None) -> TBSystem:
    """Cubic periodic cell with a (111) crack: atoms beyond the (111) plane
    through the centre with x < L/2 move ``opening`` along [111]/sqrt(3).
    The pattern here is a plain distance cutoff on the displaced positions."""
    rng = rng if rng is not None else np.random.default_rng(0)
    nx, ny, nz = cells
    ideal = diamond_lattice(nx, ny, nz)
    box = np.array([nx, ny, nz], dtype=np.float64) * A_SI
    periodic = np.array([True, True, True])
    nrm = np.ones(3) / np.sqrt(3.0)
    centre = box / 2
    beyond = ((ideal - centre) @ nrm > 0) & (ideal[:, 0] < box[0] / 2)
    pos = ideal.copy()
    pos[beyond] += opening * nrm
    pairs, trans = neighbour_pairs(pos, box, periodic, cutoff)
    meta = dict(cells=tuple(cells), opening=opening, cutoff=cutoff, n_moved=int(beyond.sum()))
    return _assemble(name, pos, box, periodic, pairs, trans, rng, meta, params)
