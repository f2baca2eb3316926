"""Bitwise reproducibility: the same inputs and options give the same bits,
for the full and projected carries, both precisions, the reductions to
charges and band energy, and the batched solve under different schedules
(concurrent streams, graph chunks)."""
import numpy as np
import pytest

from synth import configs
from synth.grids import trapezoid_weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    return api.Context(0)


@pytest.mark.parametrize("prec,carry", [("fp64", "full"), ("mixed", "full"), ("fp64", "projected"),
                                        ("mixed", "projected")])
def test_solve_twice_bitwise(ctx, prec, carry):
    from paper_1002_1202_amd import api
    print(f"case: determinism {prec} {carry}", flush=True)
    c = configs.si_small(cells=(3, 3, 2), n_shift=24, eta=0.1, n_rhs=70, seed=51)
    s, z, rhs = c["system"], c["z"], c["rhs"]
    pair, _ = api.pair_from_system(ctx, s)
    kw = dict(tol=1e-10, precision=prec, carry=carry)
    if carry == "projected":
        kw["proj"] = rhs[:, None]
    a = api.solve(ctx, pair, z, rhs=rhs, **kw)
    b = api.solve(ctx, pair, z, rhs=rhs, **kw)
    assert a.outer_iters == b.outer_iters and a.inner_iters == b.inner_iters
    if carry == "full":
        assert np.array_equal(a.G_cols, b.G_cols)
    else:
        assert np.array_equal(a.G_proj, b.G_proj)
    assert np.array_equal(a.res, b.res)
    w = trapezoid_weights(z)
    q1, e1, eb1, _ = api.mulliken_band(ctx, pair, z, w, rhs, tol=1e-10, precision=prec)
    q2, e2, eb2, _ = api.mulliken_band(ctx, pair, z, w, rhs, tol=1e-10, precision=prec)
    assert np.array_equal(q1, q2) and np.array_equal(e1, e2) and eb1 == eb2


def test_batched_schedules_bitwise(ctx):
    from paper_1002_1202_amd import api
    print("case: batched determinism under schedules", flush=True)
    cases = [configs.si_small(cells=(3, 2, 2), seed=52, n_shift=20, n_rhs=70),
             configs.water_small(n_mol=20, seed=53, n_shift=16, n_rhs=30),
             configs.si_small(cells=(2, 2, 2), seed=54, n_shift=12, n_rhs=20)]
    probs = []
    for c in cases:
        pair, _ = api.pair_from_system(ctx, c["system"])
        probs.append(dict(pair=pair, z=c["z"], rhs=c["rhs"], w=trapezoid_weights(c["z"])))
    runs = [api.solve_batched(ctx, probs, tol=1e-10, precision="mixed", **kw)
            for kw in (dict(), dict(batch_streams=1), dict(batch_streams=3, graph_iters=1))]
    for i, outs in enumerate(runs[1:]):
        for a, b in zip(runs[0], outs):
            # the iteration count is reported in whole graph chunks
            if i == 0:
                assert a["outer_iters"] == b["outer_iters"]
            assert bool((a["G_jj"] == b["G_jj"]).all())
            assert bool((a["q"] == b["q"]).all()) and bool((a["e"] == b["e"]).all())
