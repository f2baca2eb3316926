"""torch.autograd glue for the band energy, the Mulliken charges and the
ASED pair.

``BandEnergy`` runs one shifted solve with the z-derivative carry in its
forward (E_band together with dE/dH and dE/dS, the backward reusing the same
shifted solver); its backward only scales the stored gradients by the
incoming scalar.  ``MullikenCharges`` returns the charges of listed orbitals;
its backward puts the forward's H, S back into the pair (which other calls
may have changed meanwhile), solves for G e_a and G S e_a and contracts them
with the incoming charge gradient on the pattern (the general charge-loss
adjoint).
``AsedPair`` builds S, H on the device from positions and maps (dE/dH,
dE/dS) to dE/dpos with the library's VJP kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class BandEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, Hval, Sval, gctx, pair, z, w, opts):
        pair.set_values(Hval.detach().contiguous(), Sval.detach().contiguous())
        dH = torch.zeros_like(Hval)
        dS = torch.zeros_like(Sval)
        _, _, E, info = api.band_energy_vjp(gctx, pair, z, w, 1.0, dH, dS, **opts)
        fctx.save_for_backward(dH, dS)
        fctx.info = info
        return torch.tensor(E, dtype=torch.float64, device=Hval.device)

    @staticmethod
    def backward(fctx, gE):
        dH, dS = fctx.saved_tensors
        return gE * dH, gE * dS, None, None, None, None, None


class MullikenCharges(torch.autograd.Function):
    @staticmethod
    def forward(fctx, Hval, Sval, gctx, pair, z, w, orbs, opts):
        H = Hval.detach().contiguous()
        S = Sval.detach().contiguous()
        pair.set_values(H, S)
        q, _, _, info = api.mulliken_band(gctx, pair, z, w, orbs, **opts)
        # the pair is shared: another forward may change its values before
        # this backward runs, so the values of this forward are kept
        fctx.save_for_backward(H, S)
        fctx.gctx, fctx.pair, fctx.z, fctx.w, fctx.orbs, fctx.opts = gctx, pair, z, w, orbs, opts
        fctx.info = info
        return torch.from_numpy(q).to(Hval.device)

    @staticmethod
    def backward(fctx, gq):
        H, S = fctx.saved_tensors
        fctx.pair.set_values(H, S)
        qbar = gq.detach().cpu().numpy().astype(np.float64)
        shape = (fctx.pair.nnzb, fctx.pair.block, fctx.pair.block)
        dH = torch.zeros(shape, dtype=torch.float64, device=gq.device)
        dS = torch.zeros_like(dH)
        opts = {k: v for k, v in fctx.opts.items() if k != "carry"}
        api.charge_vjp(fctx.gctx, fctx.pair, fctx.z, fctx.w, fctx.orbs, qbar, dH=dH, dS=dS, **opts)
        return dH, dS, None, None, None, None, None, None


class AsedPair(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pos, gctx, pair, system, scale):
        p = pos.detach().cpu().numpy().astype(np.float64)
        api.ased_build(gctx, pair, system, scale, positions=p)
        H, S = api.pair_values_device(pair)
        fctx.gctx, fctx.pair, fctx.system, fctx.scale, fctx.p = gctx, pair, system, scale, p
        fctx.pos_device = pos.device
        return H, S

    @staticmethod
    def backward(fctx, gH, gS):
        F = api.ased_vjp(fctx.gctx, fctx.pair, fctx.system, fctx.scale, gH.contiguous(), gS.contiguous(),
                         positions=fctx.p)
        g = torch.from_numpy(-F).to(fctx.pos_device)
        return g, None, None, None, None


def mulliken_charges(gctx, pair, system, pos, z, w, orbs, scale, **opts):
    """Mulliken charges q_a(pos) of the orbitals ``orbs`` with autograd
    through the ASED pair (scale c held fixed)."""
    H, S = AsedPair.apply(pos, gctx, pair, system, scale)
    return MullikenCharges.apply(H, S, gctx, pair, z, w, np.asarray(orbs, dtype=np.int64), opts)


def band_energy(gctx, pair, system, pos, z, w, scale, **opts):
    """E_band(pos) with autograd through the ASED pair (scale c held fixed)."""
    H, S = AsedPair.apply(pos, gctx, pair, system, scale)
    return BandEnergy.apply(H, S, gctx, pair, z, w, opts)
