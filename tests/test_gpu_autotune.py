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
    best = autotune.tune_solve(ctx, pair, z, rhs, tol=1e-10, force=True)
    assert best in autotune.KNOBS_FULL
    data = json.loads(cache.read_text())
    key = autotune.shape_key(pair.block, pair.n, len(rhs), len(z), "fp64", "full")
    assert data[key]["opts"] == best
    assert any(np.isfinite(t["ms_per_iter"]) for t in data[key]["trials"])
    # second call: from the cache
    assert autotune.tune_solve(ctx, pair, z, rhs, tol=1e-10) == best
    sub = rhs[:6]
    res = api.solve(ctx, pair, z, rhs=sub, tol=1e-11, **best)
    S, H, _ = oased.dense_pair(s)
    X = ogreen.solve_dense(H, S, z, sub)
    assert float(np.abs(res.G_cols - X).max() / np.abs(X).max()) < 1e-9
