"""Reuse of cached device blocks.  Blocks of 64 MiB and more (here the
shifted vectors x^k and p^k, K x R x N complex each) are kept after a call
and handed to later calls of the same or a smaller size, still holding the
earlier call's values.  Results must not depend on that: a repeated solve is
bit-identical to the first (the kernels reduce in a fixed order), a smaller
solve in between agrees with the dense LU, and so does a solve after the
cache was handed back."""
import numpy as np
import pytest

from oracle import ased as oased, green as ogreen
from synth import configs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_cached_blocks_do_not_change_results():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    print("case: si512 K=64 R=64, cached x^k/p^k blocks (134 MB each)", flush=True)
    ctx = api.Context(0)
    c = configs.si_small(cells=(4, 4, 4), n_shift=64, eta=0.2, n_rhs=64, seed=21)
    s = c["system"]
    z, rhs = c["z"], c["rhs"]
    pair, _ = api.pair_from_system(ctx, s)
    S, H, _ = oased.dense_pair(s)
    sample = np.array([0, 31, 47])
    X = ogreen.solve_dense(H, S, z[sample], rhs)

    g1 = api.solve(ctx, pair, z, rhs=rhs, tol=1e-12).G_cols
    assert rel(g1[sample], X) < 1e-10
    # 48 shifts: the 100 MB requests take the 134 MB blocks of the first call
    r2 = api.solve(ctx, pair, z[:48], rhs=rhs, tol=1e-12, fuse_steps=8)
    assert r2.converged.all()
    assert rel(r2.G_cols[sample], X) < 1e-10
    g3 = api.solve(ctx, pair, z, rhs=rhs, tol=1e-12).G_cols
    print(f"  repeat max |diff| {np.abs(g3 - g1).max():.1e}", flush=True)
    np.testing.assert_array_equal(g3, g1)
    api.release_cache(ctx)
    g4 = api.solve(ctx, pair, z, rhs=rhs, tol=1e-12).G_cols
    np.testing.assert_array_equal(g4, g1)
