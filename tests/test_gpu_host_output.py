"""G columns returned in host memory.  Copies of 256 MiB and more go through
pinned staging buffers (three of 256 MiB, refilled while host threads drain
them); the host result must equal the device result bit for bit, for one
chunk plus a ragged tail and for more chunks than buffers."""
import numpy as np
import pytest

from synth import configs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K", [160, 448])
def test_host_output_equals_device_output(K):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    c = configs.si_small(cells=(4, 4, 4), n_shift=K, eta=0.2, n_rhs=64, seed=24)
    s = c["system"]
    nbytes = K * 64 * s.n * 16
    print(f"case: si512 K={K} R=64, G to host {nbytes / 2**20:.0f} MiB", flush=True)
    ctx = api.Context(0)
    pair, _ = api.pair_from_system(ctx, s)
    dev = api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-10, out="device")
    host = api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-10, out="host")
    assert isinstance(host.G_cols, np.ndarray) and host.G_cols.nbytes == nbytes
    np.testing.assert_array_equal(host.G_cols, dev.G_cols.cpu().numpy())
    api.release_cache(ctx)
    again = api.solve(ctx, pair, c["z"], rhs=c["rhs"], tol=1e-10, out="host")
    np.testing.assert_array_equal(again.G_cols, host.G_cols)
