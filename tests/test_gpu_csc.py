"""GPU parity of the charge-self-consistent term (Sec. 2.2, eq. Hap-CSC) and
the self-consistency loop against the CPU oracle.  Every case prints its
name before it runs."""
import numpy as np
import pytest

from oracle import ased as oased, csc as ocsc, spectral as ospec
from synth import configs
from synth.csc import hubbard_u
from synth.grids import shift_grid, trapezoid_weights

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    return api.Context(0)


def _cases():
    return [configs.water_small(n_mol=6, n_rhs=4)["system"],
            configs.si_small(cells=(2, 2, 2), n_shift=4, sigma=0.1)["system"]]


def test_csc_potential_and_hamiltonian(ctx):
    from paper_1002_1202_amd import api
    for s in _cases():
        print(f"case: csc potential/hamiltonian {s.name} atoms={s.n_atoms} B={s.block}", flush=True)
        pair, _ = api.pair_from_system(ctx, s)
        U = hubbard_u(s)
        cs = api.Csc(ctx, pair, s, U)
        G = ocsc.gamma_matrix(s, U)
        dq = np.random.default_rng(5).normal(scale=0.3, size=s.n_atoms)
        V = cs.potential(dq)
        assert rel(V, G @ dq) < 1e-13
        H0, S0 = pair.values()
        cs.hamiltonian(pair, H0, dq)
        H1, S1 = pair.values()
        np.testing.assert_array_equal(S1, S0)
        Sd, Hd, _ = oased.dense_pair(s)
        ref = oased.gather_blocks(s, ocsc.hamiltonian(Sd, Hd, G @ dq, s.orb_atom))
        assert rel(H1, ref) < 1e-13
        # zero charges give back H0
        cs.hamiltonian(pair, H0, np.zeros(s.n_atoms))
        np.testing.assert_array_equal(pair.values()[0], H0)


def _water_scc(n_mol):
    s = configs.water_small(n_mol=n_mol, n_rhs=4)["system"]
    S, H0, _ = oased.dense_pair(s)
    ev, _ = ospec.eig_pencil(H0, S)
    nocc = int(round(s.valence.sum() / 2))
    ef = 0.5 * (ev[nocc - 1] + ev[nocc])
    z = shift_grid(-60.0, ef, 128, 0.5)
    return s, S, H0, z, trapezoid_weights(z)


@pytest.mark.parametrize("n_mol,history,beta", [(4, 4, 0.2), (8, 4, 0.2), (4, 0, 0.05)])
def test_scc_loop_vs_oracle(ctx, n_mol, history, beta):
    from paper_1002_1202_amd import api
    s, S, H0, z, w = _water_scc(n_mol)
    print(f"case: scc water{n_mol} history={history} beta={beta}", flush=True)
    U = hubbard_u(s)
    G = ocsc.gamma_matrix(s, U)
    dq_ref, q_ref, eb_ref, it_ref, res_ref = ocsc.scc(s, S, H0, G, z, w, beta=beta, tol=1e-9, max_iter=1000,
                                                      history=history)
    assert res_ref <= 1e-9
    pair, _ = api.pair_from_system(ctx, s)
    cs = api.Csc(ctx, pair, s, U)
    out = cs.scc(pair, z, w, s.valence, beta=beta, history=history, scc_tol=1e-9, max_iter=1000, tol=1e-12)
    print(f"  iterations gpu {out['iterations']} oracle {it_ref}; residual {out['residual']:.1e}; "
          f"|dq - ref| {np.abs(out['dq'] - dq_ref).max():.1e}", flush=True)
    assert out["status"] == 0 and out["residual"] <= 1e-9
    # both stop within 1e-9 of the same fixed point
    np.testing.assert_allclose(out["dq"], dq_ref, atol=2e-8)
    np.testing.assert_allclose(out["q_orb"], q_ref, atol=2e-8)
    assert out["e_band"] == pytest.approx(eb_ref, rel=1e-8)
    # the pair keeps H0 + H^CSC(dq)
    ref = oased.gather_blocks(s, ocsc.hamiltonian(S, H0, G @ out["dq"], s.orb_atom))
    assert rel(pair.values()[0], ref) < 1e-12


def test_csc_errors(ctx):
    from paper_1002_1202_amd import api, _lib
    s = configs.water_small(n_mol=4, n_rhs=4)["system"]
    print("case: csc argument errors", flush=True)
    pair, _ = api.pair_from_system(ctx, s)
    U = hubbard_u(s)
    U[1] = 0.0
    with pytest.raises(_lib.GscError):
        api.Csc(ctx, pair, s, U)


@pytest.mark.parametrize("n_mol", [4, 24])
def test_scc_neutral_vs_oracle(ctx, n_mol):
    """The loop with the Fermi level set each iteration by charge
    neutrality (trapezoid weights truncated at E_F) against the oracle's
    loop: the same charges, E_F and band energy, and sum dq = 0."""
    from paper_1002_1202_amd import api
    s = configs.water_small(n_mol=n_mol, n_rhs=4)["system"]
    S, H0, _ = oased.dense_pair(s)
    z = shift_grid(-60.0, 5.0, 128, 0.5)
    print(f"case: neutral scc water{n_mol} N={s.n}", flush=True)
    U = hubbard_u(s)
    G = ocsc.gamma_matrix(s, U)
    dq_ref, q_ref, eb_ref, it_ref, res_ref, ef_ref = ocsc.scc(s, S, H0, G, z, None, beta=0.2, tol=1e-9,
                                                              max_iter=300, history=6, neutral=True)
    assert res_ref <= 1e-9
    pair, _ = api.pair_from_system(ctx, s)
    cs = api.Csc(ctx, pair, s, U)
    out = cs.scc(pair, z, None, s.valence, beta=0.2, history=6, scc_tol=1e-9, max_iter=300, neutral=True,
                 tol=1e-12)
    print(f"  iterations gpu {out['iterations']} oracle {it_ref}; E_F {out['e_fermi']:.6f} vs {ef_ref:.6f}; "
          f"|dq - ref| {np.abs(out['dq'] - dq_ref).max():.1e}; sum dq {out['dq'].sum():.1e}", flush=True)
    assert out["status"] == 0 and out["residual"] <= 1e-9
    np.testing.assert_allclose(out["dq"], dq_ref, atol=2e-8)
    np.testing.assert_allclose(out["q_orb"], q_ref, atol=2e-8)
    assert out["e_fermi"] == pytest.approx(ef_ref, abs=1e-8)
    assert out["e_band"] == pytest.approx(eb_ref, rel=1e-8)
    assert abs(out["dq"].sum()) < 1e-8
