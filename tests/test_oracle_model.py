"""Pins of the step-by-step shifted COCG model (Sec. 3.3) against the LU
definition, textbook special cases and brute force.  CPU only."""
import numpy as np
import pytest

from oracle import ased, green, shifted_cocg as sc
from synth import configs


@pytest.fixture(scope="module")
def case():
    c = configs.si_small(cells=(2, 2, 2), n_shift=12, eta=0.1)
    S, H, _ = ased.dense_pair(c["system"])
    j = int(c["rhs"][0])
    b = np.zeros(S.shape[0])
    b[j] = 1.0
    X = green.solve_dense(H, S, c["z"], [j])[:, 0, :]
    return c["z"], S, H, b, j, X


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_model_matches_lu(case):
    z, S, H, b, j, X = case
    r = sc.solve(H, S, z, b, tol=1e-13)
    assert r.converged.all()
    assert rel(r.x, X) < 1e-11


def test_printed_pi_sign_fails(case):
    """The sign printed in eq. Shift:pi does not reproduce the shifted
    systems; the derived sign does (previous test)."""
    z, S, H, b, j, X = case
    r = sc.solve(H, S, z, b, tol=1e-13, pi_sign=-1.0, max_iter=400)
    assert rel(r.x, X) > 1e-3


def test_seed_independence_and_forced_switches(case):
    z, S, H, b, j, X = case
    for seed in (0, 6, len(z) - 1):
        assert rel(sc.solve(H, S, z, b, tol=1e-13, seed=seed).x, X) < 1e-11
    r = sc.solve(H, S, z, b, tol=1e-13, force_switch=(3, 10, 50, 51))
    assert r.switches >= 4
    assert rel(r.x, X) < 1e-11


def test_shifted_iterates_equal_independent_cocg(case):
    """Collinear residual theorem: the n-th shifted iterate equals the n-th
    iterate of an independent S-preconditioned COCG run on that shift."""
    z, S, H, b, j, X = case
    n = 8
    r = sc.solve(H, S, z, b, tol=1e-30, max_iter=n, inner_tol=1e-15, seed=2)
    for k in (0, 5, 11):
        xs = sc.cocg_single(z[k] * S - H, S, b, n)
        assert rel(r.x[k], xs[-1]) < 1e-10


def test_identity_overlap_is_textbook_cocg():
    """S = I: the method reduces to plain (unpreconditioned) COCG and
    terminates in at most N steps on an N = 10 problem."""
    rng = np.random.default_rng(1)
    A = rng.normal(size=(10, 10))
    H = 0.5 * (A + A.T)
    S = np.eye(10)
    z = np.array([-1.0 + 0.5j, 0.3 + 0.5j, 2.0 + 0.5j])
    b = rng.normal(size=10)
    r = sc.solve(H, S, z, b, tol=1e-12, max_iter=40)
    X = green.solve_dense(H, S, z, B_dense=b[:, None])[:, 0, :]
    assert rel(r.x, X) < 1e-9
    assert r.iters <= 14


def test_projected_carry_with_restart(case):
    z, S, H, b, j, X = case
    Cm = np.zeros((3, S.shape[0]))
    Cm[0, j] = 1.0
    Cm[1] = S[j]
    Cm[2, (j + 9) % S.shape[0]] = 1.0
    r = sc.solve(H, S, z, b, tol=1e-13, carry="projected", proj=Cm)
    assert r.restarts >= 1
    assert rel(r.g, X @ Cm.T) < 1e-11


def test_derivative_carry_is_minus_gsg(case):
    z, S, H, b, j, X = case
    GSG = np.stack([np.linalg.inv(zk * S - H) @ S @ np.linalg.inv(zk * S - H)[:, j] for zk in z])
    r = sc.solve(H, S, z, b, tol=1e-13, deriv=True)
    assert rel(-r.dx, GSG) < 1e-9
    Cm = np.zeros((2, S.shape[0]))
    Cm[0, j] = 1.0
    Cm[1, (j + 3) % S.shape[0]] = 1.0
    rp = sc.solve(H, S, z, b, tol=1e-13, carry="projected", proj=Cm, deriv=True)
    assert rp.restarts >= 1
    assert rel(-rp.dg, GSG @ Cm.T) < 1e-9


def test_inner_cg_tolerance():
    c = configs.si_small(cells=(1, 1, 1))
    S, _, _ = ased.dense_pair(c["system"])
    r = np.random.default_rng(0).normal(size=S.shape[0]) * (1 + 1j)
    y, k = sc.inner_cg(S, r, 1e-12)
    assert np.linalg.norm(S @ y - r) <= 1e-12 * np.linalg.norm(r)
    assert k <= S.shape[0]
