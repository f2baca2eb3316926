"""Failure modes forced from the host, each a numerical condition that the
library detects and reports (no kernel faults or hangs): the iteration cap
(GSC_NOT_CONVERGED with every output, flag and residual written), an
overlap that is not positive definite (the inner CG sees d^H S d <= 0:
GSC_E_S_NOT_SPD), a NaN in H (GSC_E_NAN from the scalar controller) and a
malformed block pattern (GSC_E_ARG before any device work)."""
import numpy as np
import pytest

from oracle import ased as oased, green as ogreen
from synth import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    return api.Context(0)


@pytest.mark.parametrize("prec,carry", [("fp64", "full"), ("mixed", "projected")])
def test_iteration_cap_reports_not_converged(ctx, prec, carry):
    from paper_1002_1202_amd import _lib, api
    print(f"case: max_iter 3 {prec} {carry}", flush=True)
    c = configs.si_small(cells=(2, 2, 2), n_shift=16, eta=0.05, n_rhs=8, seed=61)
    s, z, rhs = c["system"], c["z"], c["rhs"]
    pair, _ = api.pair_from_system(ctx, s)
    kw = dict(carry=carry, proj=rhs[:, None]) if carry == "projected" else {}
    res = api.solve(ctx, pair, z, rhs=rhs, tol=1e-10, max_iter=3, precision=prec, **kw)
    assert res.status == _lib.GSC_NOT_CONVERGED
    assert res.outer_iters == 3
    assert not res.converged.all()
    assert np.all(np.isfinite(res.res)) and np.all(res.res[~res.converged] > 1e-10)
    # the flags follow the residuals, and the iterates written are finite
    assert np.array_equal(res.converged, res.res <= 1e-10)
    out = res.G_cols if carry == "full" else res.G_proj
    assert np.all(np.isfinite(out))
    # the same call with the default cap converges to the plain definition
    full = api.solve(ctx, pair, z, rhs=rhs, tol=1e-12, precision=prec)
    S, H, _ = oased.dense_pair(s)
    X = ogreen.solve_dense(H, S, z, rhs)
    assert full.status == 0
    assert float(np.abs(full.G_cols - X).max() / np.abs(X).max()) < 1e-10


def test_overlap_not_positive_definite(ctx):
    from paper_1002_1202_amd import _lib, api
    print("case: S negative definite", flush=True)
    c = configs.si_small(cells=(1, 1, 1), n_shift=4, n_rhs=4, seed=62)
    s = c["system"]
    pair, _ = api.pair_from_system(ctx, s)
    H, S = pair.values()
    pair.set_values(H, -S)
    with pytest.raises(_lib.GscError) as ei:
        api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-10)
    assert ei.value.status == -5, ei.value


def test_nan_in_hamiltonian(ctx):
    from paper_1002_1202_amd import _lib, api
    print("case: NaN in H", flush=True)
    c = configs.si_small(cells=(1, 1, 1), n_shift=4, n_rhs=4, seed=63)
    s = c["system"]
    pair, _ = api.pair_from_system(ctx, s)
    H, S = pair.values()
    H = H.copy()
    H.reshape(-1)[0] = np.nan
    pair.set_values(H, S)
    for carry in ("full", "projected"):
        kw = dict(carry=carry, proj=np.asarray(c["rhs"])[:, None]) if carry == "projected" else {}
        with pytest.raises(_lib.GscError) as ei:
            api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-10, **kw)
        assert ei.value.status == -6, (carry, ei.value)


def test_malformed_pattern_rejected(ctx):
    from paper_1002_1202_amd import _lib, api
    print("case: malformed block patterns", flush=True)
    s = configs.si_small(cells=(1, 1, 1), n_shift=4, n_rhs=4, seed=64)["system"]
    rowptr, colidx = s.rowptr.copy(), s.colidx.copy()
    bad_order = colidx.copy()
    bad_order[[0, 1]] = bad_order[[1, 0]]            # unsorted inside block row 0
    bad_range = colidx.copy()
    bad_range[-1] = s.nb                              # column block out of range
    keep = np.ones(len(colidx), bool)                 # block row 0 without its diagonal block
    keep[rowptr[0]:rowptr[1]] = colidx[rowptr[0]:rowptr[1]] != 0
    rp2 = rowptr.copy()
    rp2[1:] -= np.cumsum(~keep)[rowptr[1:] - 1]
    for name, (rp, ci) in {"unsorted": (rowptr, bad_order), "out of range": (rowptr, bad_range),
                           "missing diagonal": (rp2, colidx[keep])}.items():
        with pytest.raises(_lib.GscError) as ei:
            api.Pair(ctx, s.block, rp, ci)
        assert ei.value.status == -1, name
