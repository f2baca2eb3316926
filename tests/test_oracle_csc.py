"""Pins of the charge-self-consistent oracle (Sec. 2.2, eq. Hap-CSC) against
facts fixed by the mathematics: symmetry and the Coulomb limit of gamma, a
uniform potential shifting the generalised spectrum by exactly that
potential, zero charges leaving H unchanged, and the mixing loop's fixed
point agreeing with an independent root finder."""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from oracle import ased, csc, spectral
from synth import configs
from synth.csc import hubbard_u
from synth.grids import shift_grid, trapezoid_weights

from test_oracle_pins import dimer_system


def test_gamma_symmetric_onsite_and_coulomb_limit():
    c = configs.water_small(n_mol=6, n_rhs=4)
    s = c["system"]
    U = hubbard_u(s)
    G = csc.gamma_matrix(s, U)
    np.testing.assert_allclose(G, G.T, rtol=1e-14)
    np.testing.assert_allclose(np.diag(G), U, rtol=1e-14)
    # hard atoms (U -> infinity): the interaction becomes e^2 / r
    Gc = csc.gamma_matrix(s, U * 1e9)
    d = s.positions[:, None, :] - s.positions[None, :, :]
    r = np.sqrt((d ** 2).sum(-1))
    same_mol = (np.arange(s.n_atoms)[:, None] // 3) == (np.arange(s.n_atoms)[None, :] // 3)
    off = same_mol & ~np.eye(s.n_atoms, dtype=bool)        # intra-molecule pairs, no translation
    import scipy.constants as sc
    e2 = sc.e / (4 * np.pi * sc.epsilon_0 * 1e-10)          # e^2/(4 pi eps0) in eV * Angstrom (CODATA)
    np.testing.assert_allclose(Gc[off] * r[off], e2, rtol=1e-6)
    # finite hardness screens the interaction, more at short range
    assert (G[off] < Gc[off]).all()


def test_dimer_gamma_decreases_with_distance():
    U = np.array([6.7, 6.7])
    g = [csc.gamma_matrix(dimer_system(r=r), U)[0, 1] for r in (2.0, 2.5, 3.0, 4.0)]
    assert all(a > b for a, b in zip(g, g[1:]))


def test_uniform_potential_shifts_spectrum():
    c = configs.si_small(cells=(1, 1, 1), n_shift=4)
    s = c["system"]
    S, H0, _ = ased.dense_pair(s)
    v0 = 0.37
    H = csc.hamiltonian(S, H0, np.full(s.n_atoms, v0), s.orb_atom)
    e0 = scipy.linalg.eigh(H0, S, eigvals_only=True)
    e1 = scipy.linalg.eigh(H, S, eigvals_only=True)
    np.testing.assert_allclose(e1, e0 + v0, atol=1e-11)
    np.testing.assert_array_equal(csc.hamiltonian(S, H0, np.zeros(s.n_atoms), s.orb_atom), H0)
    # any potential keeps H symmetric and touches only the stored pattern
    V = np.random.default_rng(3).normal(size=s.n_atoms)
    Hv = csc.hamiltonian(S, H0, V, s.orb_atom)
    np.testing.assert_allclose(Hv, Hv.T, atol=1e-13)
    np.testing.assert_array_equal(Hv[S == 0], H0[S == 0])


def _water_scc_case(n_mol):
    c = configs.water_small(n_mol=n_mol, n_rhs=4)
    s = c["system"]
    S, H0, _ = ased.dense_pair(s)
    ev, _ = spectral.eig_pencil(H0, S)
    nocc = int(round(s.valence.sum() / 2))
    ef = 0.5 * (ev[nocc - 1] + ev[nocc])          # mid-gap of the neutral system
    z = shift_grid(-60.0, ef, 128, 0.5)
    return s, S, H0, z, trapezoid_weights(z)


def test_mixing_fixed_point_matches_root_finder():
    s, S, H0, z, w = _water_scc_case(4)
    G = csc.gamma_matrix(s, hubbard_u(s))
    dq, q, eb, it, res = csc.scc(s, S, H0, G, z, w, beta=0.2, tol=1e-11, max_iter=200, history=4)
    assert res <= 1e-11 and it < 200
    F = lambda x: csc.charge_response(s, S, H0, G, z, w, x)[0] - x   # noqa: E731
    root = scipy.optimize.root(F, np.zeros(s.n_atoms), tol=1e-13)
    assert root.success
    np.testing.assert_allclose(dq, root.x, atol=1e-9)
    # plain linear mixing with a small step reaches the same fixed point
    dq2, _, _, it2, res2 = csc.scc(s, S, H0, G, z, w, beta=0.05, tol=1e-11, max_iter=1000, history=0)
    assert res2 <= 1e-11
    np.testing.assert_allclose(dq2, root.x, atol=1e-9)
    # charge flows from the hydrogens to the oxygen of every molecule
    assert (dq[0::3] > 0).all() and (dq[1::3] < 0).all() and (dq[2::3] < 0).all()


def test_truncated_weights_integrate_lines_exactly():
    """The weights truncated at E_F integrate any function that is linear
    between the samples exactly from E_0 to E_F (closed form for 1 and E on
    a non-uniform grid), reduce to the full trapezoid rule at the top of the
    grid, vanish below it and are continuous through the samples."""
    rng = np.random.default_rng(5)
    E = np.sort(rng.uniform(-30.0, 5.0, 40))
    for ef in np.concatenate([rng.uniform(E[0], E[-1], 25), E[[3, 17, 39]]]):
        w = csc.truncated_weights(E, ef)
        assert w @ np.ones_like(E) == pytest.approx(ef - E[0], abs=1e-12)
        assert w @ E == pytest.approx(0.5 * (ef * ef - E[0] ** 2), abs=1e-10)
        a, b = rng.normal(size=2)
        j = np.searchsorted(E, ef, side="right") - 1
        if j < len(E) - 1:   # a piecewise-linear f: integral segment by segment
            f = a * E + b * np.abs(E - E[j])
            fe = np.interp(ef, E, f)
            ref = np.trapezoid(f[:j + 1], E[:j + 1]) + 0.5 * (ef - E[j]) * (f[j] + fe)
            assert w @ f == pytest.approx(ref, abs=1e-10)
    z = shift_grid(-20.0, 5.0, 33, 0.1)
    np.testing.assert_allclose(csc.truncated_weights(z.real, z.real[-1]), trapezoid_weights(z), atol=1e-14)
    assert not csc.truncated_weights(E, E[0] - 1.0).any()
    for k in (5, 20):
        lo = csc.truncated_weights(E, E[k] - 1e-12)
        hi = csc.truncated_weights(E, E[k] + 1e-12)
        np.testing.assert_allclose(lo, hi, atol=1e-10)


def test_fermi_level_matches_root_finder():
    """Bisection for the neutral E_F agrees with Brent's method on the same
    electron count, on a water system's actual (S G)_aa traces."""
    s, S, H0, _, _ = _water_scc_case(3)
    z = shift_grid(-60.0, 5.0, 200, 0.3)
    from oracle import green
    X = green.solve_dense(H0, S, z, np.arange(s.n))
    t = np.einsum("ij,kji->ki", S, X).imag.sum(axis=1)
    ne = float(s.valence.sum())
    ef = csc.fermi_level(z.real, t, ne)
    ref = scipy.optimize.brentq(lambda e: csc.electron_count(z.real, t, e) - ne, z.real[0], z.real[-1],
                                xtol=1e-14)
    assert ef == pytest.approx(ref, abs=1e-10)
    assert csc.electron_count(z.real, t, ef) == pytest.approx(ne, abs=1e-9)
    with pytest.raises(ValueError):
        csc.fermi_level(z.real, t, 10 * ne)


def test_neutral_scc_fixed_point_matches_root_finder():
    """The loop with E_F set by neutrality converges to the root of the
    neutral charge map (an independent solver) and its charges sum to the
    valence count (sum dq = 0)."""
    s, S, H0, _, _ = _water_scc_case(4)
    z = shift_grid(-60.0, 5.0, 160, 0.5)
    G = csc.gamma_matrix(s, hubbard_u(s))
    dq, q, eb, it, res, ef = csc.scc(s, S, H0, G, z, None, beta=0.2, tol=1e-11, max_iter=300, history=4,
                                     neutral=True)
    assert res <= 1e-11
    assert abs(dq.sum()) < 1e-9 and q.sum() == pytest.approx(s.valence.sum(), abs=1e-9)
    F = lambda x: csc.charge_response_neutral(s, S, H0, G, z, x)[0] - x   # noqa: E731
    root = scipy.optimize.root(F, np.zeros(s.n_atoms), tol=1e-13)
    assert root.success
    np.testing.assert_allclose(dq, root.x, atol=1e-8)
    assert z.real[0] < ef < z.real[-1]
