"""Parity at the benchmark's full size (si4096: N = 16384, 256 shifts,
256 right-hand sides, FP64, tol 1e-10, the launch configuration bench.py
times).  The dense oracle cannot factor 256 matrices of this size in a test,
so sampled outputs are checked one by one against what the oracle computes
cheaply from its own, independently built S and H: the true residual
||e_j - (z_k S - H) x||/||e_j|| of sampled columns, and the complex symmetry
G_ij(z) = G_ji(z) between right-hand sides of the set."""
import numpy as np
import pytest

from oracle import ased as oased, green as ogreen
from synth import configs

pytestmark = pytest.mark.gpu


def test_si4096_sampled_residuals_and_symmetry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    cfg = configs.si4096()
    s, z, rhs = cfg["system"], cfg["z"], cfg["rhs"]
    print(f"case: si4096 full size N={s.n} K={len(z)} R={len(rhs)}", flush=True)
    ctx = api.Context(0)
    pair, scale = api.pair_from_system(ctx, s)
    res = api.solve(ctx, pair, z, rhs=rhs, out="device", tol=1e-10)
    print(f"  iters={res.outer_iters} switches={res.switches} conv={res.converged.mean():.3f}", flush=True)
    assert res.converged.all()
    Sb, Hb, c0 = oased.pair_blocks(s)
    assert abs(scale - c0) <= 1e-13 * c0
    S, H = ogreen.sparse_matrices(s, Sb, Hb)
    rng = np.random.default_rng(0)
    ks = rng.choice(len(z), 8, replace=False)
    rs = rng.choice(len(rhs), 8, replace=False)
    worst = 0.0
    for k in ks:
        for r in rs:
            x = res.G_cols[k, r].cpu().numpy()
            b = np.zeros(s.n, complex)
            b[rhs[r]] = 1.0
            rr = np.linalg.norm(b - (z[k] * (S @ x) - H @ x))
            worst = max(worst, rr)
    print(f"  max sampled true residual = {worst:.2e}", flush=True)
    assert worst < 1e-8
    # complex symmetry between right-hand sides i, j of the set
    pos = {int(o): i for i, o in enumerate(rhs)}
    G = res.G_cols[ks].cpu().numpy()
    sym = 0.0
    for a in range(0, len(rhs), 17):
        for b_ in range(3, len(rhs), 29):
            i, j = int(rhs[a]), int(rhs[b_])
            gij = G[:, pos[j], i]
            gji = G[:, pos[i], j]
            # the forward error is bounded relative to the solution's scale,
            # not to one (possibly tiny) element
            scale_ = np.abs(G[:, [pos[i], pos[j]], :]).max()
            sym = max(sym, float(np.abs(gij - gji).max() / scale_))
    print(f"  max |G_ij - G_ji| / max|G| = {sym:.2e}", flush=True)
    assert sym < 1e-9
