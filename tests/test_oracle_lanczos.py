"""Pins of the generalised Lanczos oracle (Sec. 3.2, eqs. 1.13 and 1.18)
against facts fixed by the mathematics: the hand-derived dimer, exactness at
full Krylov dimension, moment matching, S-orthonormality of the basis, the
orthogonal-basis special case, and agreement with LU at convergence."""
import json
import os

import numpy as np
import pytest

from oracle import ased, green, lanczos
from synth import configs

from test_oracle_pins import GOLD, dimer_system

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _pencil(n, seed, s_off=0.15):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    H = (A + A.T) / 2
    P = rng.normal(size=(n, n)) * s_off / n
    S = np.eye(n) + (P + P.T) / 2
    assert np.linalg.eigvalsh(S).min() > 0.5
    return H, S


def test_dimer_closed_form():
    """Two orbitals: two steps are exact, and G_11 = (z - eps_2)/det(zS - H)
    with det(zS - H) the hand-derived quadratic of the golden file."""
    g = json.load(open(os.path.join(GOLD, "dimer_b1.json")))
    q = g["expected"]["pencil_quadratic"]
    eps = g["inputs"]["eps"]
    S, H, _ = ased.dense_pair(dimer_system())
    z = np.array([-15.0 + 0.3j, -9.0 + 0.05j, -2.0 + 1.0j, 4.0 + 0.2j])
    det = q["a"] * z ** 2 + q["b"] * z + q["c"]
    for j, other in ((0, 1), (1, 0)):
        a, b, vj = lanczos.lanczos(H, S, j, 2)
        assert len(a) == 2
        np.testing.assert_allclose(lanczos.continued_fraction(z, a, b, vj), (z - eps[other]) / det, rtol=1e-12)


def test_full_dimension_equals_lu():
    H, S = _pencil(12, 3)
    z = np.linspace(-3, 3, 7) + 0.2j
    for j in (0, 5, 11):
        a, b, vj = lanczos.lanczos(H, S, j, 12)
        g = lanczos.continued_fraction(z, a, b, vj)
        ref = green.solve_dense(H, S, z, [j])[:, 0, j]
        np.testing.assert_allclose(g, ref, rtol=1e-9)


def test_moments_match_the_operator_powers():
    """v_j [T^p]_00 = e_j^T (S^{-1}H)^p S^{-1} e_j for p < 2m: the defining
    property of m Lanczos steps in the S-product (a Euclidean product, a
    wrong a_n or b_n breaks it)."""
    c = configs.si_small(cells=(2, 2, 2), n_shift=4, eta=0.1)
    S, H, _ = ased.dense_pair(c["system"])
    m, j = 8, 13
    a, b, vj = lanczos.lanczos(H, S, j, m)
    T = lanczos.tridiagonal(a, b)
    scale = np.abs(np.linalg.eigvals(np.linalg.solve(S, H))).max()
    w = np.linalg.solve(S, np.eye(len(S))[:, j])
    Tp = np.eye(m)
    for p in range(2 * m):
        ref = w[j]
        assert vj * Tp[0, 0] == pytest.approx(ref, rel=1e-9, abs=1e-12 * scale ** p)
        w = np.linalg.solve(S, H @ w)
        Tp = Tp @ T


def test_basis_is_s_orthonormal_and_three_term():
    H, S = _pencil(40, 7)
    m = 12
    a, b, vj, U = lanczos.lanczos(H, S, 3, m, return_basis=True)
    np.testing.assert_allclose(U.T @ S @ U, np.eye(m), atol=1e-10)
    T = lanczos.tridiagonal(a, b)
    M = np.linalg.solve(S, H)
    # M U = U T except in the last column (which couples to u^m)
    np.testing.assert_allclose((M @ U)[:, :m - 1], (U @ T)[:, :m - 1], atol=1e-10)
    assert (b[1:] > 0).all()


def test_orthogonal_basis_special_case():
    """S = I: the plain symmetric Lanczos process; at full dimension the
    eigenvalues of T are those of H."""
    H, _ = _pencil(10, 11)
    a, b, vj = lanczos.lanczos(H, np.eye(10), 2, 10)
    assert vj == pytest.approx(1.0)
    np.testing.assert_allclose(np.linalg.eigvalsh(lanczos.tridiagonal(a, b)), np.linalg.eigvalsh(H),
                               atol=1e-9)


def test_converges_to_lu_on_silicon():
    c = configs.si_small(cells=(2, 2, 2), n_shift=16, eta=0.1)
    s = c["system"]
    S, H, _ = ased.dense_pair(s)
    rhs = c["rhs"][:3]
    ref = green.solve_dense(H, S, c["z"], rhs)
    ref = ref[:, np.arange(len(rhs)), rhs]
    g = lanczos.green_diag(H, S, c["z"], rhs, 200)
    assert np.abs(g - ref).max() / np.abs(ref).max() < 1e-8
