"""Pins of the CPU oracle against facts that do not come from the oracle
itself: a hand-derived dimer, closed forms, spectral sums, symmetry, sum
rules, finite differences and brute force.  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import ased, green, spectral, shifted_cocg as sc
from synth import configs
from synth.system import ASEDParams, TBSystem, csr_from_pairs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dimer_system(r=None, ang=0.5):
    g = json.load(open(os.path.join(GOLD, "dimer_b1.json")))["inputs"]
    p = ASEDParams(s0=g["s0"], r0=g["r0"], lam=g["lam"], kappa=g["kappa"], theta=g["theta"])
    if r is None:
        r = p.r0 + p.lam * np.log(2.0)
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    rowptr, colidx, trans, angb = csr_from_pairs(
        2, np.array([[0, 1]]), np.zeros((1, 3)), np.full((1, 1, 1), ang), np.zeros((2, 1, 1)))
    return TBSystem(name="dimer", block=1, positions=pos, orb_atom=np.arange(2),
                    eps=np.array(g["eps"]), rowptr=rowptr, colidx=colidx, trans=trans,
                    ang=angb, params=p, box=np.full(3, np.inf))


def test_dimer_golden():
    g = json.load(open(os.path.join(GOLD, "dimer_b1.json")))["expected"]
    S, H, c = ased.dense_pair(dimer_system())
    np.testing.assert_allclose(S, g["S"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(H, g["H"], rtol=1e-14)
    assert c == pytest.approx(g["c"], rel=1e-14)
    q = g["pencil_quadratic"]
    roots = np.sort(np.roots([q["a"], q["b"], q["c"]]).real)
    eps, _ = spectral.eig_pencil(H, S)
    np.testing.assert_allclose(eps, roots, rtol=1e-13)


@pytest.fixture(scope="module")
def si_small():
    c = configs.si_small(cells=(2, 2, 2), n_shift=12, eta=0.1)
    S, H, cc = ased.dense_pair(c["system"])
    return c, S, H, cc


def test_pair_structure(si_small):
    c, S, H, cc = si_small
    s = c["system"]
    assert np.abs(S - S.T).max() < 1e-15 and np.abs(H - H.T).max() < 1e-13
    np.testing.assert_array_equal(np.diag(S), 1.0)
    np.testing.assert_allclose(np.diag(H), s.eps)
    off = np.abs(S - np.eye(s.n)).sum(1)
    assert off.max() == pytest.approx(s.params.theta, rel=1e-13)
    ev = np.linalg.eigvalsh(S)
    # Gershgorin: diag 1, off-site row sums <= theta
    assert ev.min() >= 1 - s.params.theta - 1e-12 and ev.max() <= 1 + s.params.theta + 1e-12
    # two orbitals of one atom never overlap
    for a in range(0, 8):
        blk = S[4 * a:4 * a + 4, 4 * a:4 * a + 4]
        np.testing.assert_array_equal(blk, np.eye(4))


@pytest.mark.parametrize("make", [
    lambda: configs.si_small(cells=(2, 2, 2), n_shift=2)["system"],
    lambda: configs.water_small(n_mol=24, n_shift=2)["system"],
    lambda: configs.slab_small(cells=(2, 2, 3), n_shift=2)["system"],
])
def test_sparse_assembly_matches_dense(make):
    """The CSR assembly that the full-size checks use places every stored
    block where the dense assembly (an explicit loop over blocks) puts it:
    the same entries bit for bit, both triangles, nothing summed twice."""
    s = make()
    Sb, Hb, c = ased.pair_blocks(s)
    S, H = green.sparse_matrices(s, Sb, Hb)
    Sd, Hd, cd = ased.dense_pair(s, c)
    assert cd == c
    np.testing.assert_array_equal(S.toarray(), Sd)
    np.testing.assert_array_equal(H.toarray(), Hd)
    assert S.nnz == s.nnzb * s.block ** 2


def test_green_lu_vs_spectral_and_symmetry(si_small):
    c, S, H, _ = si_small
    z = c["z"]
    rhs = np.array([0, 5, 17, 100])
    X = green.solve_dense(H, S, z, rhs)
    eps, C = spectral.eig_pencil(H, S)
    for k in range(len(z)):
        G = spectral.green_spectral(eps, C, z[k])
        np.testing.assert_allclose(X[k], G[:, rhs].T, rtol=0, atol=1e-12 * np.abs(G).max())
    # complex symmetry G_ij = G_ji from two independent solves
    Xi = green.solve_dense(H, S, z, [5, 17])
    np.testing.assert_allclose(Xi[:, 0, 17], Xi[:, 1, 5], rtol=1e-12)


def test_green_diagonal_closed_form():
    rng = np.random.default_rng(3)
    e = rng.uniform(-20, 5, 12)
    z = np.array([-3.0 + 0.1j, 1.0 + 0.05j])
    X = green.solve_dense(np.diag(e), np.eye(12), z, np.arange(12))
    for k in range(2):
        np.testing.assert_allclose(np.diagonal(X[k]), 1.0 / (z[k] - e), rtol=1e-14)


def test_green_2x2_closed_form():
    H = np.array([[-3.0, 1.2], [1.2, 0.5]])
    S = np.array([[1.0, 0.3], [0.3, 1.0]])
    z = np.array([0.7 + 0.2j])
    X = green.solve_dense(H, S, z, [0, 1])[0]
    a, b, d = z[0] * S[0, 0] - H[0, 0], z[0] * S[0, 1] - H[0, 1], z[0] * S[1, 1] - H[1, 1]
    det = a * d - b * b
    inv = np.array([[d, -b], [-b, a]]) / det
    np.testing.assert_allclose(X.T, inv, rtol=1e-14)


def test_trace_sg(si_small):
    c, S, H, _ = si_small
    z = c["z"][:3]
    n = S.shape[0]
    X = green.solve_dense(H, S, z, np.arange(n))
    eps, _ = spectral.eig_pencil(H, S)
    for k in range(3):
        tr = np.sum(S * X[k])                 # sum_a (S x^(a))_a
        assert abs(tr - np.sum(1 / (z[k] - eps))) < 1e-10 * abs(tr)


def test_mulliken_band_vs_spectral(si_small):
    c, S, H, _ = si_small
    from synth.grids import shift_grid, trapezoid_weights
    z = shift_grid(-25.0, -6.0, 60, 0.3)
    w = trapezoid_weights(z)
    orb = np.arange(S.shape[0])
    X = green.solve_dense(H, S, z, orb)
    q, e, eb = green.mulliken_band(S, X, z, w, orb)
    q2, e2, eb2 = spectral.mulliken_band_spectral(H, S, z, w, orb)
    np.testing.assert_allclose(q, q2, rtol=0, atol=1e-11)
    np.testing.assert_allclose(e, e2, rtol=0, atol=1e-10)
    assert eb == pytest.approx(eb2, rel=1e-12)
    # sum rule: sum_a q_a = 2 sum_n W(eps_n)
    eps, _ = spectral.eig_pencil(H, S)
    assert q.sum() == pytest.approx(2 * spectral.window_W(eps, z, w).sum(), rel=1e-12)


def test_sum_rule_counts_states():
    """A window far wider than the spectrum and eta much smaller than the
    grid extent: every state is counted twice (spin), sum_a q_a ~ 2N."""
    c = configs.si_small(cells=(1, 1, 1), sigma=0.0)
    S, H, _ = ased.dense_pair(c["system"])
    from synth.grids import shift_grid, trapezoid_weights
    z = shift_grid(-400.0, 400.0, 16001, 0.05)
    w = trapezoid_weights(z)
    eps, _ = spectral.eig_pencil(H, S)
    total = 2 * spectral.window_W(eps, z, w).sum()
    assert total == pytest.approx(2 * S.shape[0], rel=2e-3)


def test_gradients_lu_vs_spectral_and_fd(si_small):
    c, S, H, _ = si_small
    from synth.grids import shift_grid, trapezoid_weights
    z = shift_grid(-20.0, -6.65, 24, 0.2)
    w = trapezoid_weights(z)
    gH, gS = green.band_energy_grad_dense(H, S, z, w)
    sH, sS = spectral.band_energy_grad_spectral(H, S, z, w)
    np.testing.assert_allclose(gH, sH, rtol=0, atol=1e-10 * np.abs(sH).max())
    np.testing.assert_allclose(gS, sS, rtol=0, atol=1e-10 * np.abs(sS).max())

    def eband(Hm, Sm):
        return sum(-(2 / np.pi) * wk * zk.real * np.trace(Sm @ np.linalg.inv(zk * Sm - Hm)).imag
                   for zk, wk in zip(z, w))
    h = 1e-6
    for (b, cc) in [(0, 0), (0, 5), (3, 64)]:
        E = np.zeros_like(H)
        E[b, cc] = h
        fdH = (eband(H + E, S) - eband(H - E, S)) / (2 * h)
        fdS = (eband(H, S + E) - eband(H, S - E)) / (2 * h)
        assert fdH == pytest.approx(gH[b, cc], rel=1e-5, abs=1e-8)
        assert fdS == pytest.approx(gS[b, cc], rel=1e-5, abs=1e-8)


def test_forces_vs_fd():
    c = configs.si_small(cells=(1, 1, 1), sigma=0.08, seed=5)
    s = c["system"]
    from synth.grids import shift_grid, trapezoid_weights
    z = shift_grid(-20.0, -6.65, 16, 0.3)
    w = trapezoid_weights(z)
    S, H, cc = ased.dense_pair(s)
    gH, gS = green.band_energy_grad_dense(H, S, z, w)
    F = ased.forces(s, ased.gather_blocks(s, gH), ased.gather_blocks(s, gS), cc)

    def eband(pos):
        s2 = TBSystem(**{**s.__dict__, "positions": pos})
        S2, H2, _ = ased.dense_pair(s2, c=cc)
        return sum(-(2 / np.pi) * wk * zk.real * np.trace(S2 @ np.linalg.inv(zk * S2 - H2)).imag
                   for zk, wk in zip(z, w))
    h = 1e-5
    for atom, ax in [(0, 0), (3, 2), (6, 1)]:
        p1 = s.positions.copy()
        p2 = s.positions.copy()
        p1[atom, ax] += h
        p2[atom, ax] -= h
        fd = -(eband(p1) - eband(p2)) / (2 * h)
        assert fd == pytest.approx(F[atom, ax], rel=1e-5, abs=1e-7)
    # Newton's third law: internal forces sum to zero
    assert np.abs(F.sum(0)).max() < 1e-10


def test_dimer_force_fd():
    z = np.linspace(-20, -8, 9) + 0.2j
    w = np.full(9, 1.5)
    s = dimer_system()
    S, H, cc = ased.dense_pair(s)
    gH, gS = green.band_energy_grad_dense(H, S, z, w)
    F = ased.forces(s, ased.gather_blocks(s, gH), ased.gather_blocks(s, gS), cc)

    def eband(r):
        S2, H2, _ = ased.dense_pair(dimer_system(r=r), c=cc)
        return sum(-(2 / np.pi) * wk * zk.real * np.trace(S2 @ np.linalg.inv(zk * S2 - H2)).imag
                   for zk, wk in zip(z, w))
    r0 = s.positions[1, 0]
    fd = -(eband(r0 + 1e-6) - eband(r0 - 1e-6)) / 2e-6
    assert F[1, 0] == pytest.approx(fd, rel=1e-6)
