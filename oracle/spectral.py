"""Closed forms from the generalised eigen-decomposition H c = eps S c with
S-normalised eigenvectors (c_n^T S c_n = 1).  These pin the LU oracle: they
reach G, the charges, the band energy and its gradients by a completely
different route (spectral sums instead of factorisations).

    G(z)        = sum_n c_n c_n^T / (z - eps_n)
    Tr(S G(z))  = sum_n 1 / (z - eps_n)
    q_a         = 2 sum_n W(eps_n) (S c_n)_a c_{n,a}
    e_a         = 2 sum_n F(eps_n) (S c_n)_a c_{n,a}
    E_band      = 2 sum_n F(eps_n)
    dE/dH       = 2 sum_n F'(eps_n) c_n c_n^T
    dE/dS       = -2 sum_n F'(eps_n) eps_n c_n c_n^T
with the Lorentzian-broadened window functions of the quadrature
    W(e) = (1/pi) sum_k w_k eta_k / ((E_k - e)^2 + eta_k^2)
    F(e) = (1/pi) sum_k w_k E_k eta_k / ((E_k - e)^2 + eta_k^2).
The gradient lines follow from d eps_n / dH_bc = c_nb c_nc and
d eps_n / dS_bc = -eps_n c_nb c_nc for the symmetric-definite pencil.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def eig_pencil(H, S):
    eps, C = scipy.linalg.eigh(H, S)
    return eps, C


def green_spectral(eps, C, z):
    return (C / (z - eps)[None, :]) @ C.T


def window_W(eps, z, w):
    E, eta = z.real, z.imag
    return (1.0 / np.pi) * np.sum(w[:, None] * eta[:, None]
                                  / ((E[:, None] - eps[None, :]) ** 2 + eta[:, None] ** 2), 0)


def window_F(eps, z, w):
    E, eta = z.real, z.imag
    return (1.0 / np.pi) * np.sum(w[:, None] * E[:, None] * eta[:, None]
                                  / ((E[:, None] - eps[None, :]) ** 2 + eta[:, None] ** 2), 0)


def window_Fprime(eps, z, w):
    E, eta = z.real, z.imag
    dd = E[:, None] - eps[None, :]
    return (1.0 / np.pi) * np.sum(w[:, None] * E[:, None] * eta[:, None] * 2.0 * dd
                                  / (dd ** 2 + eta[:, None] ** 2) ** 2, 0)


def mulliken_band_spectral(H, S, z, w, orb_idx):
    eps, C = eig_pencil(H, S)
    pop = (S @ C) * C                         # (S c_n)_a c_{n,a}
    Wn = window_W(eps, z, w)
    Fn = window_F(eps, z, w)
    q = 2.0 * pop[orb_idx] @ Wn
    e = 2.0 * pop[orb_idx] @ Fn
    return q, e, 2.0 * Fn.sum()


def band_energy_grad_spectral(H, S, z, w):
    eps, C = eig_pencil(H, S)
    Fp = window_Fprime(eps, z, w)
    gH = 2.0 * (C * Fp[None, :]) @ C.T
    gS = -2.0 * (C * (Fp * eps)[None, :]) @ C.T
    return gH, gS
