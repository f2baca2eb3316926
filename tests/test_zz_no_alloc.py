"""The allocation-free product gsc_spmm_noalloc (temporaries in a fixed
per-device scratch array) against gsc_spmm, which allocates its own, and
against the oracle's dense product: two calls in a row, the second with a
smaller input, a ragged column count (padded copies in the scratch) and a
multiple of 64 (in place), and the size check that rejects a call the
scratch cannot hold."""
import ctypes as C

import numpy as np
import pytest

from oracle import ased as oased
from synth import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    return api.Context(0)


def _case(ctx, c, nrhs, seed):
    import torch
    from paper_1002_1202_amd import api
    s = c["system"]
    pair, _ = api.pair_from_system(ctx, s)
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(s.n, nrhs)) + 1j * rng.normal(size=(s.n, nrhs))
    alpha = rng.uniform(-20, 5, nrhs) + 1j * rng.uniform(0.01, 0.2, nrhs)
    Xd = torch.from_numpy(X).to("cuda:0")
    return s, pair, X, Xd, alpha


def test_noalloc_matches_allocating_product(ctx):
    import torch
    from paper_1002_1202_amd import api
    cases = [(configs.si_small(cells=(3, 3, 3), seed=51), 70),     # ragged: padded copies
             (configs.water_small(n_mol=20, seed=52), 64)]          # smaller, in place
    for (c, nrhs), seed in zip(cases, (1, 2)):
        s, pair, X, Xd, alpha = _case(ctx, c, nrhs, seed)
        print(f"case: spmm_noalloc {s.name} N={s.n} nrhs={nrhs}", flush=True)
        Y0 = api.spmm(ctx, pair, Xd, alpha)
        Y1 = torch.full_like(Xd, complex(np.nan, np.nan))
        out = api.spmm_noalloc(ctx, pair, Xd, alpha, Y=Y1)
        assert out is Y1
        torch.cuda.synchronize()
        a, b = Y1.cpu().numpy(), Y0.cpu().numpy()
        assert np.isfinite(a).all()
        diff = float(np.abs(a - b).max() / np.abs(b).max())
        S, H, _ = oased.dense_pair(s)
        ref = alpha[None, :] * (S @ X) - H @ X
        err = float(np.abs(a - ref).max() / np.abs(ref).max())
        print(f"  vs gsc_spmm {diff:.2e}, vs dense oracle {err:.2e}", flush=True)
        assert diff <= 1e-15
        assert err < 1e-13


def test_noalloc_rejects_what_the_scratch_cannot_hold(ctx):
    import torch
    from paper_1002_1202_amd import _lib, api
    c = configs.si_small(cells=(6, 6, 6), seed=53)
    s = c["system"]
    pair, _ = api.pair_from_system(ctx, s)
    nrhs = 1000                       # 2 padded copies of N x 1024 complex: > 64 MiB
    print(f"case: spmm_noalloc too large N={s.n} nrhs={nrhs}", flush=True)
    X = torch.zeros((s.n, nrhs), dtype=torch.complex128, device="cuda:0")
    alpha = np.ones(nrhs, np.complex128)
    with pytest.raises(RuntimeError, match="scratch"):
        api.spmm_noalloc(ctx, pair, X, alpha)
    # the context is still usable, and a call that fits works
    Xs = torch.ones((s.n, 64), dtype=torch.complex128, device="cuda:0")
    Y = api.spmm_noalloc(ctx, pair, Xs, np.ones(64))
    ref = api.spmm(ctx, pair, Xs, np.ones(64))
    assert float((Y - ref).abs().max()) <= 1e-15 * float(ref.abs().max())
