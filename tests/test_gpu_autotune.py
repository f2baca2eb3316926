"""The launch-shape autotuner: it times the candidates on the real problem,
caches the winner per shape class, answers the next call from the cache, and
the tuned options give the same solution.  Every case prints its name."""
import json
import os

import numpy as np
import pytest

from oracle import ased as oased, green as ogreen
from synth import configs

pytestmark = pytest.mark.gpu


def test_tune_solve_caches_and_keeps_parity(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api, autotune
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("GSC_AUTOTUNE_CACHE", str(cache))
    c = configs.si_small(cells=(4, 4, 4), n_shift=16, eta=0.1, n_rhs=64, seed=31)
    s, z, rhs = c["system"], c["z"], c["rhs"]
    print(f"case: autotune N={s.n} K={len(z)} R={len(rhs)}", flush=True)
    ctx = api.Context(0)
    pair, _ = api.pair_from_system(ctx, s)
    space = {"fuse_steps": [0, 8], "cheb_block": [0, 64], "row_groups": [0, 64]}
    best = autotune.tune_solve(ctx, pair, z, rhs, tol=1e-10, space=space, force=True)
    assert all(k in space and v in space[k][1:] for k, v in best.items())
    data = json.loads(cache.read_text())
    key = autotune.shape_key(pair.block, pair.n, len(rhs), len(z), "fp64", "full")
    assert data[key]["opts"] == best
    # one trial per option set of the coordinate search (1 + one per knob);
    # a trial whose two lengths do not separate counts as infinitely slow
    assert len(data[key]["trials"]) == 4
    assert any(np.isfinite(t["ms_per_iter"]) for t in data[key]["trials"])
    # second call: from the cache
    assert autotune.tune_solve(ctx, pair, z, rhs, tol=1e-10, space=space) == best
    sub = rhs[:6]
    res = api.solve(ctx, pair, z, rhs=sub, tol=1e-11, **best)
    S, H, _ = oased.dense_pair(s)
    X = ogreen.solve_dense(H, S, z, sub)
    assert float(np.abs(res.G_cols - X).max() / np.abs(X).max()) < 1e-9


def test_tune_batched_tile_shapes_cache_and_parity(tmp_path, monkeypatch):
    """tune_batched searches tile and launch shapes of a small uneven batch
    (graph chunk, concurrent jobs, rhs tile, row groups), stores the winner
    under the batch's shape class, answers the next call from the cache, and
    the batch solved with the tuned shapes matches the oracle at the FP64
    bar."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api, autotune
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("GSC_AUTOTUNE_CACHE", str(cache))
    cases = [configs.si_small(cells=(3, 3, 2), seed=41, n_shift=24, n_rhs=150),
             configs.si_small(cells=(2, 2, 2), seed=42, n_shift=16, n_rhs=40),
             configs.water_small(n_mol=24, seed=43, n_shift=20, n_rhs=60)]
    ctx = api.Context(0)
    probs = []
    for c in cases:
        pair, _ = api.pair_from_system(ctx, c["system"])
        probs.append(dict(pair=pair, z=c["z"], rhs=c["rhs"]))
    print(f"case: tune_batched {[p['pair'].n for p in probs]}", flush=True)
    space = {"graph_iters": [0, 1], "batch_streams": [0, 2], "rhs_tile": [0, 64], "row_groups": [0, 64]}
    best = autotune.tune_batched(ctx, probs, precision="fp64", tol=1e-10, t1=4, t2=24, space=space, force=True)
    print(f"  best {best}", flush=True)
    assert all(k in space and v in space[k][1:] for k, v in best.items())
    data = json.loads(cache.read_text())
    key = autotune.batch_key(probs, "fp64")
    assert data[key]["opts"] == best
    assert len(data[key]["trials"]) == 5
    assert any(np.isfinite(t["ms_per_iter"]) for t in data[key]["trials"])
    assert autotune.tune_batched(ctx, probs, precision="fp64", space=space) == best
    outs = api.solve_batched(ctx, probs, tol=1e-12, **best)
    for c, o in zip(cases, outs):
        s, z, rhs = c["system"], c["z"], c["rhs"]
        S, H, _ = oased.dense_pair(s)
        X = ogreen.solve_dense(H, S, z, rhs)
        g0 = X[:, np.arange(len(rhs)), rhs]
        err = float(np.abs(o["G_jj"].cpu().numpy() - g0).max() / np.abs(g0).max())
        print(f"  N={s.n} R={len(rhs)} iters={o['outer_iters']} err={err:.2e}", flush=True)
        assert o["converged"].all() and err < 1e-10
