"""Pins of the charge-loss gradient oracle: it reduces to the (separately
pinned) band-energy gradient for Q = I with weights w_k E_k, and matches
central finite differences of the Mulliken charges entry by entry."""
import numpy as np
import pytest

from oracle import ased, green
from synth import configs


@pytest.fixture(scope="module")
def case():
    c = configs.water_small(n_mol=3, n_rhs=4, n_shift=6, eta=0.4)
    s = c["system"]
    S, H, _ = ased.dense_pair(s)
    z = c["z"]
    w = np.linspace(0.3, 1.1, len(z))
    return s, S, H, z, w


def test_reduces_to_band_energy_gradient(case):
    s, S, H, z, w = case
    gH, gS = green.charge_grad_dense(H, S, z, w * z.real, np.arange(s.n), np.ones(s.n))
    eH, eS = green.band_energy_grad_dense(H, S, z, w)
    np.testing.assert_allclose(gH, eH, atol=1e-12)
    np.testing.assert_allclose(gS, eS, atol=1e-12)


def test_finite_differences(case):
    s, S, H, z, w = case
    rng = np.random.default_rng(2)
    orbs = np.array([0, 3, 7, 10, 15])
    qbar = rng.normal(size=len(orbs))
    gH, gS = green.charge_grad_dense(H, S, z, w, orbs, qbar)

    def loss(Hm, Sm):
        X = green.solve_dense(Hm, Sm, z, orbs)
        q, _, _ = green.mulliken_band(Sm, X, z, w, orbs)
        return float(qbar @ q)

    h = 1e-6
    for (b, c) in [(0, 1), (3, 3), (7, 2), (12, 15), (5, 11)]:
        for M, g in ((0, gH), (1, gS)):
            Ep = [H.copy(), S.copy()]
            Em = [H.copy(), S.copy()]
            Ep[M][b, c] += h
            Em[M][b, c] -= h
            fd = (loss(*Ep) - loss(*Em)) / (2 * h)
            assert fd == pytest.approx(g[b, c], rel=1e-5, abs=1e-9)
