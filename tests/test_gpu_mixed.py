"""Mixed precision (FP64 seed process; inner S-solve in complex64 Chebyshev
rounds refined by FP64 residuals) against the dense-LU oracle at the
workloads' broadening eta = 0.05 eV: G, charges and band energy within 1e-6
(1e-5 e on charges) at the workloads' tol 1e-6, at the FP64 bar at tight
tol, and the gradients of the band energy and of a charge loss."""
import numpy as np
import pytest

from oracle import ased as oased, green as ogreen
from synth import configs
from synth.grids import trapezoid_weights

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    return api.Context(0)


@pytest.fixture(scope="module")
def cases():
    out = []
    for c in (configs.si_small(cells=(3, 3, 3), n_shift=40, eta=0.05, n_rhs=70, seed=41),
              configs.water_small(n_mol=40, n_shift=40, eta=0.05, n_rhs=70, seed=42)):
        s = c["system"]
        S, H, _ = oased.dense_pair(s)
        X = ogreen.solve_dense(H, S, c["z"], c["rhs"])
        out.append((c, S, H, X))
    return out


def test_mixed_projected_and_charges_at_tol_1e6(ctx, cases):
    """G_jj (projected carry) and the Mulliken charges / band energy at tol
    1e-6: within 1e-6 of max|G_jj| and 1e-5 e; B = 4 and B = 6, 70 rhs (a
    ragged second chunk of columns)."""
    from paper_1002_1202_amd import api
    for c, S, H, X in cases:
        s, z, rhs = c["system"], c["z"], c["rhs"]
        print(f"case: mixed projected {s.name} N={s.n} tol 1e-6", flush=True)
        pair, _ = api.pair_from_system(ctx, s)
        g0 = X[:, np.arange(len(rhs)), rhs]
        res = api.solve(ctx, pair, z, rhs=rhs, tol=1e-6, precision="mixed", carry="projected",
                        proj=rhs[:, None])
        eg = rel(res.G_proj[:, :, 0], g0)
        w = trapezoid_weights(z)
        q, e, eb, info = api.mulliken_band(ctx, pair, z, w, rhs, tol=1e-6, precision="mixed")
        q0, e0, _ = ogreen.mulliken_band(S, X, z, w, rhs)
        dq = float(np.abs(q - q0).max())
        print(f"  G_jj err={eg:.2e} |dq|={dq:.2e} e err={rel(e, e0):.2e} iters={info['outer_iters']}",
              flush=True)
        assert res.status == 0 and info["status"] == 0
        assert eg < 1e-6
        assert dq < 1e-5
        assert rel(e, e0) < 1e-6


@pytest.mark.parametrize("relax", [False, True])
def test_mixed_full_carry_fp64_bar(ctx, cases, relax):
    """Full carry at tol 1e-12: whole G columns at the FP64 bar (1e-10) and
    FP64 true residuals below 1e-10, with the fixed and the relaxed inner
    tolerance (the relaxed plan changes the number of complex64 rounds as
    the shifts converge)."""
    from paper_1002_1202_amd import api
    for c, S, H, X in cases:
        s, z, rhs = c["system"], c["z"], c["rhs"]
        print(f"case: mixed full {s.name} tol 1e-12 relax={relax}", flush=True)
        pair, _ = api.pair_from_system(ctx, s)
        res = api.solve(ctx, pair, z, rhs=rhs, tol=1e-12, precision="mixed", recheck=True, inner_relax=relax)
        err = rel(res.G_cols, X)
        print(f"  err={err:.2e} res_true={res.res_true.max():.2e} iters={res.outer_iters} "
              f"inner={res.inner_iters}", flush=True)
        assert res.status == 0
        assert err < 1e-10
        assert res.res_true.max() < 1e-10


def test_mixed_deep_refinement(ctx, cases):
    """tol 1e-13 asks for an inner tolerance of 1e-15: three complex64 rounds
    per inner solve; the columns still reach the FP64 bar."""
    from paper_1002_1202_amd import api
    c, S, H, X = cases[0]
    s, z, rhs = c["system"], c["z"], c["rhs"][:20]
    print("case: mixed tol 1e-13 (three refinement rounds)", flush=True)
    pair, _ = api.pair_from_system(ctx, s)
    api.profile_enable(ctx, True)
    res = api.solve(ctx, pair, z, rhs=rhs, tol=1e-13, precision="mixed", recheck=True)
    prof = api.profile_read(ctx)
    api.profile_enable(ctx, False)
    err = rel(res.G_cols, X[:, :20])
    print(f"  err={err:.2e} res_true={res.res_true.max():.2e} cheb_mx={prof['cheb_mx'][1]} "
          f"mx_resid={prof['mx_resid'][1]}", flush=True)
    assert err < 1e-11
    assert res.res_true.max() < 1e-11
    # two residual passes per inner solve after the first (CG) solve
    assert prof["mx_resid"][1] == 2 * (res.outer_iters)
    assert prof["cheb_mx"][2] > 0 and prof["cheb_step"][1] == 0


def test_mixed_band_energy_and_charge_gradients(ctx, cases):
    """The backward paths with mixed precision at tol 1e-12: dE/dH, dE/dS
    (z-derivative carry) and a charge loss's dL/dH, dL/dS (two shifted
    solves) against the dense oracle at the FP64 bar."""
    from paper_1002_1202_amd import api
    c = configs.water_small(n_mol=12, n_shift=16, eta=0.05, seed=43)
    s, z = c["system"], c["z"]
    print(f"case: mixed gradients {s.name} N={s.n}", flush=True)
    S, H, _ = oased.dense_pair(s)
    pair, _ = api.pair_from_system(ctx, s)
    w = trapezoid_weights(z)
    dH, dS, E, _ = api.band_energy_vjp(ctx, pair, z, w, tol=1e-12, precision="mixed")
    gH, gS = ogreen.band_energy_grad_dense(H, S, z, w)
    eH = rel(dH, oased.gather_blocks(s, gH))
    eS = rel(dS, oased.gather_blocks(s, gS))
    orbs = np.array([0, 7, 20, 33, 50])
    qbar = np.array([1.0, -0.4, 0.8, 2.0, -1.5])
    cH, cS, _ = api.charge_vjp(ctx, pair, z, w, orbs, qbar, tol=1e-12, precision="mixed")
    rH, rS = ogreen.charge_grad_dense(H, S, z, w, orbs, qbar)
    print(f"  dE/dH {eH:.2e} dE/dS {eS:.2e} dL/dH {rel(cH, oased.gather_blocks(s, rH)):.2e} "
          f"dL/dS {rel(cS, oased.gather_blocks(s, rS)):.2e}", flush=True)
    assert eH < 1e-9 and eS < 1e-9
    assert rel(cH, oased.gather_blocks(s, rH)) < 1e-9
    assert rel(cS, oased.gather_blocks(s, rS)) < 1e-9


@pytest.mark.parametrize("block", [0, 128])
def test_mixed_two_column_step_and_tail(ctx, block):
    """The complex64 Chebyshev step runs 128-column pieces with two columns
    per lane and a 64-column tail with one: 150 rhs (a 192-column tile, its
    last 42 columns padding), unblocked and in column blocks of 128, against
    the dense LU at the FP64 bar."""
    from paper_1002_1202_amd import api
    c = configs.si_small(cells=(3, 3, 2), n_shift=16, eta=0.05, n_rhs=150, seed=46, vacancy_frac=0.03)
    s, z, rhs = c["system"], c["z"], c["rhs"]
    print(f"case: mixed two-column step N={s.n} R={len(rhs)} cheb_block={block}", flush=True)
    S, H, _ = oased.dense_pair(s)
    X = ogreen.solve_dense(H, S, z, rhs)
    pair, _ = api.pair_from_system(ctx, s)
    res = api.solve(ctx, pair, z, rhs=rhs, tol=1e-12, precision="mixed", cheb_block=block, recheck=True)
    print(f"  err={rel(res.G_cols, X):.2e} res_true={res.res_true.max():.2e}", flush=True)
    assert res.status == 0
    assert rel(res.G_cols, X) < 1e-10
    assert res.res_true.max() < 1e-10
