"""The five synthetic workloads, plus small replicas used by parity tests.

Each workload is seeded with ``1000 + index`` (1001 ... 1005) and returns a
plain dict: ``system`` (TBSystem), ``z`` (complex128 shifts), ``rhs`` (int64
orbital indices j of the unit right-hand sides e_j), ``tol`` and a few
workload-specific extras.  Nothing here evaluates the method.
"""
from __future__ import annotations

import itertools

import numpy as np

from .grids import rhs_atoms, shift_grid, trapezoid_weights
from .silicon import si_bulk, si_crack_111, si_slab_001
from .water import water_box


def si64(seed: int = 1001) -> dict:
    """Si diamond 2x2x2 cells (64 atoms, N = 256); 64 shifts on [-20, 5] eV,
    eta = 0.1 eV; RHS e_0 ... e_7; tol 1e-10."""
    rng = np.random.default_rng(seed)
    system = si_bulk((2, 2, 2), rng=rng, name="si64")
    return dict(name="si64", system=system, z=shift_grid(-20.0, 5.0, 64, 0.1),
                rhs=np.arange(8, dtype=np.int64), tol=1e-10, precision="fp64")


def si4096(seed: int = 1002) -> dict:
    """Si diamond 8x8x8 cells (4096 atoms, N = 16384), Gaussian displacements
    sigma = 0.05 A; 256 shifts on [-20, 5] eV, eta = 0.05 eV; 256 RHS = all
    orbitals of 64 random atoms; tol 1e-10."""
    rng = np.random.default_rng(seed)
    system = si_bulk((8, 8, 8), rng=rng, sigma=0.05, name="si4096")
    rhs = rhs_atoms(rng, system.n_atoms, 64, 4)
    return dict(name="si4096", system=system, z=shift_grid(-20.0, 5.0, 256, 0.05),
                rhs=rhs, tol=1e-10, precision="fp64")


def _near_cubic_cells(target_atoms: float):
    best = None
    for a, b, c in itertools.product(range(2, 17), repeat=3):
        if not (a <= b <= c) or c > 2 * a:
            continue
        n = 8 * a * b * c
        key = (abs(n - target_atoms), c - a)
        if best is None or key < best[0]:
            best = (key, (a, b, c))
    return best[1]


def batch32(seed: int = 1003, n_sys: int = 32, max_log2: float = 15.0) -> dict:
    """32 uneven Si systems: log2(atoms) ~ U[9, 15], near-cubic cells, vacancies
    U[0, 2%], uniaxial strain U[0, 5%]; the last one is a (111) crack.  Shifts
    K_s ~ U{128..1024} on [-20, 5] eV (eta 0.05), RHS R_s ~ U{64..512} in
    multiples of 4 (all orbitals of R_s/4 random atoms); tol 1e-6."""
    rng = np.random.default_rng(seed)
    items = []
    for s in range(n_sys):
        log2n = rng.uniform(9.0, max_log2)
        cells = _near_cubic_cells(2.0 ** log2n)
        if s == n_sys - 1:
            cube = max(cells)
            system = si_crack_111((cube, cube, cube), rng=rng, name=f"batch{s}-crack")
        else:
            system = si_bulk(cells, rng=rng, strain=rng.uniform(0.0, 0.05),
                             vacancy_frac=rng.uniform(0.0, 0.02), name=f"batch{s}")
        k = int(rng.integers(128, 1025))
        r = 4 * int(rng.integers(16, 129))
        r = min(r, 4 * system.n_atoms)
        rhs = rhs_atoms(rng, system.n_atoms, r // 4, 4)
        items.append(dict(system=system, z=shift_grid(-20.0, 5.0, k, 0.05), rhs=rhs))
    return dict(name="batch32", items=items, tol=1e-6, precision="mixed")


def slab8192(seed: int = 1004, cells=(8, 8, 16), e_fermi: float | None = None) -> dict:
    """Si (001) slab, 8x8 cells laterally x 16 thick (8192 atoms, N = 32768),
    dimer-like top layer; 512 shifts on [-20, E_F] with trapezoid weights,
    eta = 0.05 eV; all orbitals as RHS; tol 1e-10.  ``e_fermi`` is a caller
    input (default -6.65 eV)."""
    rng = np.random.default_rng(seed)
    system = si_slab_001(cells, rng=rng, name="slab%d" % (8 * np.prod(cells)))
    ef = -6.65 if e_fermi is None else e_fermi
    z = shift_grid(-20.0, ef, 512, 0.05)
    return dict(name=system.name, system=system, z=z, w=trapezoid_weights(z),
                rhs=np.arange(system.n, dtype=np.int64), tol=1e-10, e_fermi=ef,
                precision="fp64", fd_step=1e-4)


def water3000(seed: int = 1005, n_mol: int = 3000) -> dict:
    """3000 H2O at 1 g/cm^3 (N = 18000, B = 6), cutoff 6 A; 1024 shifts on
    [-40, 5] eV, eta = 0.05 eV; all orbitals as RHS; tol 1e-6."""
    rng = np.random.default_rng(seed)
    system = water_box(n_mol, rng=rng, name="water%d" % n_mol)
    return dict(name=system.name, system=system, z=shift_grid(-40.0, 5.0, 1024, 0.05),
                rhs=np.arange(system.n, dtype=np.int64), tol=1e-6, precision="mixed")


# ----------------------------------------------------------------- replicas
def si_small(cells=(2, 2, 2), seed: int = 7, sigma: float = 0.05, n_shift: int = 16,
             eta: float = 0.1, n_rhs: int = 8, e_lo=-20.0, e_hi=5.0, **kw) -> dict:
    rng = np.random.default_rng(seed)
    system = si_bulk(cells, rng=rng, sigma=sigma, name="si-small", **kw)
    n_rhs = min(n_rhs, system.n)
    rhs = np.sort(rng.choice(system.n, size=n_rhs, replace=False)).astype(np.int64)
    return dict(name="si-small", system=system, z=shift_grid(e_lo, e_hi, n_shift, eta),
                rhs=rhs, tol=1e-12)


def water_small(n_mol: int = 48, seed: int = 11, n_shift: int = 16, eta: float = 0.1,
                n_rhs: int = 12, cutoff: float = 6.0) -> dict:
    rng = np.random.default_rng(seed)
    system = water_box(n_mol, rng=rng, cutoff=cutoff, name="water-small")
    n_rhs = min(n_rhs, system.n)
    rhs = np.sort(rng.choice(system.n, size=n_rhs, replace=False)).astype(np.int64)
    return dict(name="water-small", system=system, z=shift_grid(-40.0, 5.0, n_shift, eta),
                rhs=rhs, tol=1e-12)


def slab_small(cells=(2, 2, 4), seed: int = 13, n_shift: int = 24, eta: float = 0.1) -> dict:
    rng = np.random.default_rng(seed)
    system = si_slab_001(cells, rng=rng, name="slab-small")
    z = shift_grid(-20.0, -6.65, n_shift, eta)
    return dict(name="slab-small", system=system, z=z, w=trapezoid_weights(z),
                rhs=np.arange(system.n, dtype=np.int64), tol=1e-12, e_fermi=-6.65)
