"""GPU parity of the backward: dE/dH, dE/dS against the oracle's dense
G S G form, and forces through the ASED pair against the oracle and central
finite differences."""
import numpy as np
import pytest

from oracle import ased as oased, green as ogreen
from synth import configs
from synth.grids import shift_grid, trapezoid_weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_1202_amd import api
    return api.Context(0)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("case", ["si", "water", "slab"])
def test_band_energy_vjp_vs_dense(ctx, case):
    from paper_1002_1202_amd import api
    if case == "si":
        c = configs.si_small(cells=(2, 2, 2), seed=3)
        z = shift_grid(-20.0, -6.65, 24, 0.2)
    elif case == "water":
        c = configs.water_small(n_mol=24)
        z = shift_grid(-40.0, -12.0, 24, 0.3)
    else:
        c = configs.slab_small(cells=(2, 2, 2), n_shift=24, eta=0.2)
        z = c["z"]
    s = c["system"]
    w = trapezoid_weights(z)
    print(f"case: vjp {case} N={s.n} K={len(z)}", flush=True)
    pair, scale = api.pair_from_system(ctx, s)
    dH, dS, E, info = api.band_energy_vjp(ctx, pair, z, w, tol=1e-12)
    S, H, _ = oased.dense_pair(s)
    gH, gS = ogreen.band_energy_grad_dense(H, S, z, w)
    X = ogreen.solve_dense(H, S, z, np.arange(s.n))
    _, _, E0 = ogreen.mulliken_band(S, X, z, w, np.arange(s.n))
    rH, rS = rel(dH, oased.gather_blocks(s, gH)), rel(dS, oased.gather_blocks(s, gS))
    print(f"  E={E:.10f} E0={E0:.10f} rel dH={rH:.2e} dS={rS:.2e} restarts={info['restarts']}", flush=True)
    assert abs(E - E0) <= 1e-10 * abs(E0)
    assert rH < 1e-9 and rS < 1e-9


def test_autograd_forces_vs_oracle_and_fd(ctx):
    import torch
    from paper_1002_1202_amd import api, autograd
    c = configs.si_small(cells=(1, 1, 2), sigma=0.06, seed=8)
    s = c["system"]
    z = shift_grid(-20.0, -6.65, 20, 0.25)
    w = trapezoid_weights(z)
    print(f"case: autograd forces N={s.n}", flush=True)
    pair, scale = api.pair_from_system(ctx, s)
    pos = torch.tensor(s.positions, dtype=torch.float64, requires_grad=True)
    E = autograd.band_energy(ctx, pair, s, pos, z, w, scale, tol=1e-12)
    E.backward()
    F = -pos.grad.numpy()
    S, H, cc = oased.dense_pair(s, c=scale)
    gH, gS = ogreen.band_energy_grad_dense(H, S, z, w)
    F0 = oased.forces(s, oased.gather_blocks(s, gH), oased.gather_blocks(s, gS), scale)
    print(f"  |F-F0|/|F0| = {rel(F, F0):.2e}", flush=True)
    assert rel(F, F0) < 1e-8
    # central finite differences of the GPU energy (pattern, c, angles fixed)
    h = 1e-4
    for atom, ax in [(0, 0), (5, 2), (11, 1)]:
        e = []
        for sgn in (1, -1):
            p = s.positions.copy()
            p[atom, ax] += sgn * h
            api.ased_build(ctx, pair, s, scale, positions=p)
            _, _, Eh, _ = api.band_energy_vjp(ctx, pair, z, w, tol=1e-13)
            e.append(Eh)
        fd = -(e[0] - e[1]) / (2 * h)
        print(f"  atom {atom} ax {ax}: F={F[atom, ax]:.8e} fd={fd:.8e}", flush=True)
        assert fd == pytest.approx(F[atom, ax], rel=1e-5, abs=1e-7)


def test_band_energy_vjp_slices_add_up(ctx):
    """The backward over a partition of the orbitals (three uneven slices,
    host and device gradients) adds up to the call over every orbital, and
    each slice's energy is the sum of its orbitals' e_a from the forward."""
    import torch
    from paper_1002_1202_amd import api
    c = configs.water_small(n_mol=16)
    s = c["system"]
    z = shift_grid(-40.0, -12.0, 20, 0.3)
    w = trapezoid_weights(z)
    print(f"case: vjp slices water N={s.n}", flush=True)
    pair, _ = api.pair_from_system(ctx, s)
    dH, dS, E, _ = api.band_energy_vjp(ctx, pair, z, w, tol=1e-12)
    perm = np.random.default_rng(2).permutation(s.n)
    parts = [perm[:7], perm[7:50], perm[50:]]
    shape = (pair.nnzb, pair.block, pair.block)
    sH = torch.zeros(shape, dtype=torch.float64, device="cuda:0")
    sS = torch.zeros_like(sH)
    _, e_orb, _, _ = api.mulliken_band(ctx, pair, z, w, np.arange(s.n), tol=1e-12)
    Es = 0.0
    for p in parts:
        _, _, e, _ = api.band_energy_vjp(ctx, pair, z, w, 1.0, sH, sS, orbs=p, tol=1e-12)
        assert abs(e - e_orb[p].sum()) <= 1e-9 * np.abs(e_orb[p]).sum()
        Es += e
    assert abs(Es - E) <= 1e-10 * abs(E)
    assert rel(sH.cpu().numpy(), dH) < 1e-10 and rel(sS.cpu().numpy(), dS) < 1e-10
    with pytest.raises(Exception, match="twice"):
        api.band_energy_vjp(ctx, pair, z, w, orbs=np.array([3, 5, 3]))
    with pytest.raises(Exception, match="range"):
        api.band_energy_vjp(ctx, pair, z, w, orbs=np.array([s.n]))
