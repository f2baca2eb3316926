"""GPU parity of the HIP path against the CPU oracle (dense LU and the
closed-form reductions).  Every case prints its name before it runs."""
import numpy as np
import pytest

from oracle import ased as oased, green as ogreen, shifted_cocg as omodel
from synth import configs
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


@pytest.fixture(scope="module")
def si216():
    """Si 3x3x3 cells (216 atoms, N = 864), displaced; 16 shifts; 70 rhs
    (two 64-wide waves, ragged tail)."""
    c = configs.si_small(cells=(3, 3, 3), n_shift=16, eta=0.1, n_rhs=70, seed=21)
    S, H, cc = oased.dense_pair(c["system"])
    return c, S, H, cc


def test_ased_build_matches_oracle(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, cc = si216
    s = c["system"]
    print("case: ased build si216", flush=True)
    pair, scale = api.pair_from_system(ctx, s)
    Hv, Sv = pair.values()
    Sb, Hb, _ = oased.pair_blocks(s)
    assert abs(scale - cc) <= 1e-14 * cc
    np.testing.assert_allclose(Sv, Sb, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Hv, Hb, rtol=0, atol=1e-13)


def test_ased_build_water(ctx):
    from paper_1002_1202_amd import api
    c = configs.water_small(n_mol=40)
    s = c["system"]
    print("case: ased build water40", flush=True)
    pair, scale = api.pair_from_system(ctx, s)
    Hv, Sv = pair.values()
    Sb, Hb, cc = oased.pair_blocks(s)
    assert abs(scale - cc) <= 1e-14 * cc
    np.testing.assert_allclose(Sv, Sb, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Hv, Hb, rtol=0, atol=1e-13)


def test_spmm_matches_dense(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: spmm si216 R=70", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rng = np.random.default_rng(0)
    X = rng.normal(size=(S.shape[0], 70)) + 1j * rng.normal(size=(S.shape[0], 70))
    a = rng.normal(size=70) + 1j * rng.normal(size=70)
    Y = api.spmm(ctx, pair, X, a)
    ref = (S @ X) * a[None, :] - H @ X
    assert rel(Y, ref) < 1e-14


def test_solve_full_carry_vs_lu(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: solve full carry si216 K=16 R=70 tol=1e-12", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    res = api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-12, recheck=True)
    X = ogreen.solve_dense(H, S, c["z"], c["rhs"])
    err = rel(res.G_cols, X)
    print(f"  iters={res.outer_iters} switches={res.switches} err={err:.2e} "
          f"res_true_max={res.res_true.max():.2e}", flush=True)
    assert res.status == 0 and res.converged.all()
    assert err < 1e-10
    assert res.res_true.max() < 1e-10


@pytest.mark.parametrize("m", [1, 4, 16])
def test_fused_steps_do_not_change_result(ctx, si216, m):
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print(f"case: fuse_steps={m}", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"][:20]
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, fuse_steps=m)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    assert rel(res.G_cols, X) < 1e-10


def test_seed_choice_invariance(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: seed 0 / K-1", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"][:8]
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    for seed in (0, len(c["z"]) - 1):
        res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, seed_index=seed)
        assert rel(res.G_cols, X) < 1e-10


def test_projected_carry_vs_lu(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: projected carry si216", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"]
    n = S.shape[0]
    proj = np.stack([rhs, (rhs + 7) % n, (rhs * 3 + 1) % n], 1)
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, carry="projected", proj=proj)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    ref = np.take_along_axis(X, np.broadcast_to(proj[None], (X.shape[0],) + proj.shape), axis=2)
    print(f"  iters={res.outer_iters} restarts={res.restarts} err={rel(res.G_proj, ref):.2e}", flush=True)
    assert rel(res.G_proj, ref) < 1e-10


def test_full_carry_projection_output(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: full carry with G_proj", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"][:10]
    proj = np.stack([rhs, (rhs + 1) % S.shape[0]], 1)
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, proj=proj, want_cols=False)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    ref = np.take_along_axis(X, np.broadcast_to(proj[None], (X.shape[0],) + proj.shape), axis=2)
    assert rel(res.G_proj, ref) < 1e-10


@pytest.mark.parametrize("carry", ["full", "projected"])
def test_mulliken_band_vs_oracle(ctx, carry):
    from paper_1002_1202_amd import api
    c = configs.si_small(cells=(2, 2, 2), seed=4)
    s = c["system"]
    S, H, _ = oased.dense_pair(s)
    z = shift_grid(-20.0, -6.65, 40, 0.1)
    w = trapezoid_weights(z)
    orb = np.arange(s.n)
    print(f"case: mulliken/band si64 all orbitals carry={carry}", flush=True)
    pair, _ = api.pair_from_system(ctx, s)
    q, e, eb, info = api.mulliken_band(ctx, pair, z, w, orb, tol=1e-12, carry=carry)
    X = ogreen.solve_dense(H, S, z, orb)
    q0, e0, eb0 = ogreen.mulliken_band(S, X, z, w, orb)
    print(f"  dq={np.abs(q - q0).max():.2e} de={np.abs(e - e0).max():.2e} "
          f"dEb={abs(eb - eb0) / abs(eb0):.2e}", flush=True)
    assert np.abs(q - q0).max() < 1e-10
    assert np.abs(e - e0).max() < 1e-9
    assert abs(eb - eb0) <= 1e-10 * abs(eb0)


def test_water_full_carry(ctx):
    from paper_1002_1202_amd import api
    c = configs.water_small(n_mol=40, n_rhs=20)
    s = c["system"]
    print("case: water40 B=6 full carry", flush=True)
    S, H, _ = oased.dense_pair(s)
    pair, _ = api.pair_from_system(ctx, s)
    res = api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-12)
    X = ogreen.solve_dense(H, S, c["z"], c["rhs"])
    assert rel(res.G_cols, X) < 1e-10


def test_dense_rhs_and_device_output(ctx, si216):
    import torch
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: dense rhs, device outputs", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rng = np.random.default_rng(5)
    B = rng.normal(size=(5, S.shape[0])) + 1j * rng.normal(size=(5, S.shape[0]))
    res = api.solve(ctx, pair, c["z"][:6], B=B, tol=1e-12, out="device")
    X = ogreen.solve_dense(H, S, c["z"][:6], B_dense=B.T)
    assert isinstance(res.G_cols, torch.Tensor)
    assert rel(res.G_cols.cpu().numpy(), X) < 1e-10


def test_iterates_match_model_after_few_steps(ctx):
    """With max_iter = 6 the GPU stops early (GSC_NOT_CONVERGED) and its
    iterates equal the step-by-step model's after 6 steps."""
    from paper_1002_1202_amd import api
    c = configs.si_small(cells=(2, 2, 2), n_shift=8, seed=9)
    s = c["system"]
    S, H, _ = oased.dense_pair(s)
    j = int(c["rhs"][0])
    print("case: early stop max_iter=6", flush=True)
    pair, _ = api.pair_from_system(ctx, s)
    res = api.solve(ctx, pair, c["z"], rhs=[j], tol=1e-12, max_iter=6, inner_tol=1e-15, seed_index=3)
    assert res.status == 1 and not res.converged.any()
    b = np.zeros(s.n)
    b[j] = 1.0
    m = omodel.solve(H, S, c["z"], b, tol=1e-12, max_iter=6, inner_tol=1e-15, seed=3)
    assert rel(res.G_cols[:, 0, :], m.x) < 1e-11
    np.testing.assert_allclose(res.res[:, 0], m.res, rtol=1e-9)


@pytest.mark.parametrize("tol,bar", [(1e-8, 1e-6), (1e-12, 1e-10)])
def test_mixed_precision_accuracy(ctx, si216, tol, bar):
    """Mixed precision, full carry: whole G columns against the dense LU.
    tol 1e-8 reaches 1e-6 (the recursion's tolerance is not the accuracy of
    G: at tol 1e-6 even FP64 columns are off by about 1e-5); tol 1e-12 the
    FP64 bar, with FP64 true residuals below 1e-10."""
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print(f"case: mixed precision si216 tol {tol:g}", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"][:16]
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=tol, precision="mixed", recheck=True)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    err = rel(res.G_cols, X)
    print(f"  mixed err={err:.2e} res_true_max={res.res_true.max():.2e}", flush=True)
    assert res.status == 0
    assert err < bar
    assert res.res_true.max() < 100 * tol


def test_c64_precision_floor(ctx, si216):
    """The all-complex64 seed process stalls near cond(z S - H) eps32: below
    1e-3 here, whatever tol asks."""
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print("case: complex64 seed process si216", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"][:16]
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-6, precision="c64", recheck=True)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    err = rel(res.G_cols, X)
    print(f"  c64 err={err:.2e} res_true_max={res.res_true.max():.2e}", flush=True)
    assert err < 1e-3


def test_argument_errors(ctx, si216):
    from paper_1002_1202_amd import api, _lib
    c, S, H, _ = si216
    print("case: argument errors", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    with pytest.raises(_lib.GscError) as e:
        api.solve(ctx, pair, np.array([1.0 + 0.0j]), rhs=[0])
    assert e.value.status == -1
    with pytest.raises(_lib.GscError) as e:
        api.solve(ctx, pair, c["z"], rhs=[S.shape[0]])
    assert e.value.status == -1
    s = c["system"]
    bad = s.colidx.copy()
    bad[0], bad[1] = bad[1], bad[0]
    with pytest.raises(_lib.GscError) as e:
        api.Pair(ctx, 4, s.rowptr, bad)
    assert e.value.status == -1


def test_not_spd_and_nan_detected(ctx):
    from paper_1002_1202_amd import api, _lib
    c = configs.si_small(cells=(1, 1, 1))
    s = c["system"]
    Sb, Hb, _ = oased.pair_blocks(s)
    print("case: S not SPD, NaN in H", flush=True)
    pair = api.Pair(ctx, 4, s.rowptr, s.colidx, Hb, -Sb)
    with pytest.raises(_lib.GscError) as e:
        api.solve(ctx, pair, c["z"], rhs=[0, 1])
    assert e.value.status == -5
    Hn = Hb.copy()
    Hn[0, 0, 0] = np.nan
    pair2 = api.Pair(ctx, 4, s.rowptr, s.colidx, Hn, Sb)
    with pytest.raises(_lib.GscError) as e:
        api.solve(ctx, pair2, c["z"], rhs=[0, 1])
    assert e.value.status == -6


def test_ased_vjp_matches_oracle(ctx, si216):
    from paper_1002_1202_amd import api
    c, S, H, cc = si216
    s = c["system"]
    print("case: ASED VJP forces", flush=True)
    pair, scale = api.pair_from_system(ctx, s)
    rng = np.random.default_rng(2)
    dH = rng.normal(size=(s.nnzb, 4, 4))
    dS = rng.normal(size=(s.nnzb, 4, 4))
    F = api.ased_vjp(ctx, pair, s, scale, dH, dS)
    F0 = oased.forces(s, dH, dS, cc)
    assert rel(F, F0) < 1e-12


@pytest.mark.parametrize("method", [1, 2])
def test_inner_methods(ctx, si216, method):
    """Inner S-solve by CG (1) or by the Chebyshev iteration on the Ritz
    interval of the first CG solve (2): both reach the LU solution."""
    from paper_1002_1202_amd import api
    c, S, H, _ = si216
    print(f"case: inner_method={method}", flush=True)
    pair, _ = api.pair_from_system(ctx, c["system"])
    rhs = c["rhs"][:24]
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, inner_method=method, recheck=True)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    print(f"  iters={res.outer_iters} inner={res.inner_iters} err={rel(res.G_cols, X):.2e}", flush=True)
    assert rel(res.G_cols, X) < 1e-10
    assert res.res_true.max() < 1e-10


def test_chebyshev_projected_water(ctx):
    from paper_1002_1202_amd import api
    c = configs.water_small(n_mol=40, n_rhs=16)
    s = c["system"]
    print("case: water40 projected + chebyshev", flush=True)
    S, H, _ = oased.dense_pair(s)
    pair, _ = api.pair_from_system(ctx, s)
    rhs = c["rhs"]
    proj = np.stack([rhs, (rhs + 5) % s.n], 1)
    res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, carry="projected", proj=proj, inner_method=2)
    X = ogreen.solve_dense(H, S, c["z"], rhs)
    ref = np.take_along_axis(X, np.broadcast_to(proj[None], (X.shape[0],) + proj.shape), axis=2)
    assert rel(res.G_proj, ref) < 1e-10


@pytest.mark.parametrize("carry", ["full", "projected"])
def test_ragged_tail_water_and_si(ctx, si216, carry):
    """B = 4 and B = 6 with a ragged tail of columns (70 rhs -> a second,
    partly padded 64-column chunk), both carries."""
    from paper_1002_1202_amd import api
    print(f"case: ragged tail carry={carry}", flush=True)
    for c in (si216[0], configs.water_small(n_mol=40, n_rhs=23)):
        s = c["system"]
        S, H, _ = oased.dense_pair(s)
        pair, _ = api.pair_from_system(ctx, s)
        rhs = c["rhs"][:70]
        X = ogreen.solve_dense(H, S, c["z"], rhs)
        if carry == "full":
            res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12)
            assert rel(res.G_cols, X) < 1e-10
        else:
            proj = rhs[:, None]
            res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, carry="projected", proj=proj)
            assert rel(res.G_proj[:, :, 0], X[:, np.arange(len(rhs)), rhs]) < 1e-10


@pytest.mark.parametrize("kernel,hint", [(1, 2)])
def test_chebyshev_kernel_variants(ctx, si216, kernel, hint):
    """The Chebyshev step with nontemporal streamed vectors (stream_hint 2),
    B = 4 and B = 6, a ragged column tail (70 rhs -> 2 tiles of 64), FP64
    and complex64 products."""
    from paper_1002_1202_amd import api
    print(f"case: chebyshev spmm_kernel={kernel} stream_hint={hint}", flush=True)
    for c in (si216[0], configs.water_small(n_mol=40, n_rhs=23)):
        s = c["system"]
        S, H, _ = oased.dense_pair(s)
        pair, _ = api.pair_from_system(ctx, s)
        rhs = c["rhs"][:70]
        X = ogreen.solve_dense(H, S, c["z"], rhs)
        res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, spmm_kernel=kernel, inner_method=2,
                        stream_hint=hint, recheck=True)
        print(f"  {s.name}: iters={res.outer_iters} inner={res.inner_iters} err={rel(res.G_cols, X):.2e}",
              flush=True)
        assert rel(res.G_cols, X) < 1e-10
        assert res.res_true.max() < 1e-10
        proj = rhs[:, None]
        res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, spmm_kernel=kernel, inner_method=2,
                        stream_hint=hint, carry="projected", proj=proj)
        assert rel(res.G_proj[:, :, 0], X[:, np.arange(len(rhs)), rhs]) < 1e-10
        resm = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-6, spmm_kernel=kernel, inner_method=2,
                         stream_hint=hint, precision="c64")
        print(f"  c64 err={rel(resm.G_cols, X):.2e}", flush=True)
        assert rel(resm.G_cols, X) < 1e-3


@pytest.mark.parametrize("block", [64, 128])
def test_chebyshev_column_blocks(ctx, block):
    """The inner Chebyshev solve run one column block at a time (all steps of
    a block, then the next; a ragged last block), full and projected carry,
    B = 4 and B = 6, against the dense LU and the unblocked solve."""
    from paper_1002_1202_amd import api
    print(f"case: chebyshev column blocks of {block}", flush=True)
    cases = [configs.si_small(cells=(3, 3, 3), n_shift=8, eta=0.2, n_rhs=300, seed=31),
             configs.water_small(n_mol=60, n_rhs=200, n_shift=8)]
    for c in cases:
        s = c["system"]
        S, H, _ = oased.dense_pair(s)
        pair, _ = api.pair_from_system(ctx, s)
        rhs = c["rhs"]
        X = ogreen.solve_dense(H, S, c["z"], rhs)
        res = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, inner_method=2, cheb_block=block)
        ref = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, inner_method=2)
        print(f"  {s.name} R={len(rhs)}: err={rel(res.G_cols, X):.2e} "
              f"vs unblocked {rel(res.G_cols, ref.G_cols):.2e}", flush=True)
        assert rel(res.G_cols, X) < 1e-10
        assert rel(res.G_cols, ref.G_cols) < 1e-11
        resp = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-12, inner_method=2, cheb_block=block,
                         carry="projected", proj=rhs[:, None])
        assert rel(resp.G_proj[:, :, 0], X[:, np.arange(len(rhs)), rhs]) < 1e-10
        # mixed and complex64 precision: the same arithmetic per column,
        # blocked or not
        resm = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-8, inner_method=2, cheb_block=block,
                         precision="mixed")
        refm = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-8, inner_method=2, precision="mixed")
        assert rel(resm.G_cols, refm.G_cols) < 1e-12
        assert rel(resm.G_cols, X) < 1e-6
        resc = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-6, inner_method=2, cheb_block=block,
                         precision="c64")
        refc = api.solve(ctx, pair, c["z"], rhs=rhs, tol=1e-6, inner_method=2, precision="c64")
        assert rel(resc.G_cols, refc.G_cols) < 1e-12
        assert rel(resc.G_cols, X) < 1e-3
