"""torch.autograd glue for the band energy and the ASED pair.

``BandEnergy`` runs one shifted solve with the z-derivative carry in its
forward (E_band together with dE/dH and dE/dS, the backward reusing the same
shifted solver); its backward only scales the stored gradients by the
incoming scalar.  ``AsedPair`` builds S, H on the device from positions and
maps (dE/dH, dE/dS) to dE/dpos with the library's VJP kernels.
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


def band_energy(gctx, pair, system, pos, z, w, scale, **opts):
    """E_band(pos) with autograd through the ASED pair (scale c held fixed)."""
    H, S = AsedPair.apply(pos, gctx, pair, system, scale)
    return BandEnergy.apply(H, S, gctx, pair, z, w, opts)
