"""Step-by-step model of the generalised shifted COCG method (Sec. 3.3),
FP64 / complex128, one right-hand side at a time, written in the order of
the section: the seed recurrences (eqs. CGp:p, CGp:x, CGp:r with r' = S^{-1} r),
the shift equation with the scalar pi recurrence (eq. Shift:pi), the collinear
residual theorem (eq. Collinear), the inner CG for S^{-1} r and seed switching.

Conventions (readings of the section, all listed in the design notes):
  * the system family is A(z) = z S - H, i.e. the section's sigma is -z and its
    solution is the negative of ours; delta_k = z_k - z_s;
  * products inside alpha and beta are the *unconjugated* S-bilinear form,
    so (r', r')_S = r'^T r and (p, (S^{-1}A) p)_S = p^T A p;
  * pi_{n+1} = (1 + alpha_n delta) pi_n + (alpha_n beta_{n-1}/alpha_{n-1})(pi_n - pi_{n-1});
    the second term's sign is the one obtained by eliminating p from the seed
    recurrences (the printed sign does not reproduce the shifted systems);
  * alpha^k_n = alpha_n pi_n / pi_{n+1},  beta^k_{n-1} = (pi_{n-1}/pi_n)^2 beta_{n-1},
    p^k_n = r'_n / pi_n + beta^k_{n-1} p^k_{n-1},  x^k_{n+1} = x^k_n + alpha^k_n p^k_n;
  * a shift is frozen once ||r_n|| / (|pi_n| ||b||) <= tol;
  * seed switching keeps the Krylov history: when the seed converges the
    least-converged active shift becomes the seed and the seed quantities are
    rescaled by its pi (the shifted iterates are unchanged by the rescale);
  * with projected carry only c_m^T x^k and c_m^T p^k are kept, and a
    converged seed triggers a collinear restart (new right-hand side r, each
    shift weighted by its accumulated 1/pi);
  * the z-derivative of every shifted iterate is carried alongside
    (d/dz of the recurrences at a fixed seed process); -dx/dz = G S G b.

This is test infrastructure: it is never called by the product path.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def inner_cg(S, r, tol: float, max_iter: int = 1000):
    """Hermitian CG for S y = r (S real symmetric positive definite), zero
    start, stop at ||r - S y|| <= tol ||r||.  Returns y and the step count."""
    y = np.zeros_like(r)
    res = r.copy()
    d = res.copy()
    rr = np.vdot(res, res).real
    stop = (tol * np.linalg.norm(r)) ** 2
    k = 0
    while rr > stop and k < max_iter:
        w = S @ d
        a = rr / np.vdot(d, w).real
        y = y + a * d
        res = res - a * w
        rr_new = np.vdot(res, res).real
        d = res + (rr_new / rr) * d
        rr = rr_new
        k += 1
    return y, k


def default_seed(z) -> int:
    """Shift whose real part is nearest the middle of the grid (ties: lower k)."""
    e = np.asarray(z).real
    mid = 0.5 * (e.min() + e.max())
    return int(np.argmin(np.abs(e - mid)))


@dataclass
class Result:
    x: np.ndarray | None            # (K, N) full carry
    g: np.ndarray | None            # (K, M) projections c_m^T x_k
    dx: np.ndarray | None = None    # (K, N) d x_k / d z_k
    dg: np.ndarray | None = None    # (K, M)
    res: np.ndarray | None = None   # (K,) recursive residual estimates at exit
    converged: np.ndarray | None = None
    iters: int = 0
    active_shift_iters: int = 0     # sum over iterations of the number of active shifts
    inner_iters: int = 0
    switches: int = 0
    restarts: int = 0
    seeds: list = field(default_factory=list)


def solve(H, S, z, b, tol: float = 1e-10, max_iter: int = 2000, inner_tol=None,
          seed=None, carry: str = "full", proj=None, deriv: bool = False,
          force_switch: tuple = (), pi_sign: float = +1.0) -> Result:
    """Run the method for one right-hand side ``b`` and all shifts ``z``.

    ``proj`` (M, N) holds the projection vectors c_m for carry="projected".
    ``force_switch``: iteration numbers after which the seed is switched even
    if it has not converged (tests the invariance of the iterates).
    ``pi_sign`` = -1 runs the printed sign of eq. Shift:pi (for a negative test).
    """
    z = np.asarray(z, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    K, N = z.shape[0], b.shape[0]
    if inner_tol is None:
        inner_tol = max(1e-2 * tol, 1e-15)
    s = default_seed(z) if seed is None else int(seed)
    full = carry == "full"
    C = None if proj is None else np.asarray(proj, dtype=np.complex128)

    def project(v):
        return C @ v

    out = Result(x=np.zeros((K, N), complex) if full else None,
                 g=np.zeros((K, C.shape[0]), complex) if C is not None else None)
    X = out.x
    P = np.zeros((K, N), complex) if full else None
    G = out.g
    Hp = np.zeros_like(G) if G is not None else None
    if deriv:
        out.dx = np.zeros((K, N), complex) if full else None
        out.dg = np.zeros_like(G) if G is not None else None
        dP = np.zeros((K, N), complex) if full else None
        dHp = np.zeros_like(G) if G is not None else None
        dpi = np.zeros(K, complex)
        dpi_prev = np.zeros(K, complex)
    omega = np.ones(K, complex)          # collinear-restart weights
    domega = np.zeros(K, complex)

    bnorm = np.linalg.norm(b)
    r = b.copy()
    rp, k_in = inner_cg(S, r, inner_tol)
    out.inner_iters += k_in
    p = rp.copy()
    rho = rp @ r
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    pi = np.ones(K, complex)
    pi_prev = np.ones(K, complex)
    active = np.ones(K, bool)
    res_final = np.ones(K)
    out.seeds.append(s)

    for n in range(max_iter):
        zs = z[s]
        # seed: q = A_s p, alpha = (r', r')_S / (p, S^{-1} A_s p)_S
        q = zs * (S @ p) - H @ p
        alpha = rho / (p @ q)
        # shift equation: pi recurrence and the shifted coefficients
        delta = z - zs
        lead = 1.0 + alpha * delta
        tail = alpha * beta_prev / alpha_prev
        pi_next = lead * pi + pi_sign * tail * (pi - pi_prev)
        alpha_k = alpha * pi / pi_next
        beta_k = (pi_prev / pi) ** 2 * beta_prev
        if deriv:
            dpi_next = alpha * pi + lead * dpi + pi_sign * tail * (dpi - dpi_prev)
            dalpha_k = alpha * (dpi * pi_next - pi * dpi_next) / pi_next ** 2
            dbeta_k = 2.0 * beta_prev * (pi_prev / pi) * (dpi_prev * pi - pi_prev * dpi) / pi ** 2
        # shifted vectors (only the active shifts move)
        a = active
        out.active_shift_iters += int(a.sum())
        if full:
            P_old = P[a].copy()
            P[a] = rp[None, :] / pi[a, None] + beta_k[a, None] * P[a]
            X[a] += (omega[a] * alpha_k[a])[:, None] * P[a]
            if deriv:
                dP[a] = (-rp[None, :] * (dpi[a] / pi[a] ** 2)[:, None]
                         + dbeta_k[a, None] * P_old + beta_k[a, None] * dP[a])
                out.dx[a] += (domega[a] * alpha_k[a])[:, None] * P[a] + omega[a, None] * (
                    dalpha_k[a, None] * P[a] + alpha_k[a, None] * dP[a])
        if G is not None:
            crp = project(rp)
            H_old = Hp[a].copy()
            Hp[a] = crp[None, :] / pi[a, None] + beta_k[a, None] * Hp[a]
            G[a] += (omega[a] * alpha_k[a])[:, None] * Hp[a]
            if deriv:
                dHp[a] = (-crp[None, :] * (dpi[a] / pi[a] ** 2)[:, None]
                          + dbeta_k[a, None] * H_old + beta_k[a, None] * dHp[a])
                out.dg[a] += (domega[a] * alpha_k[a])[:, None] * Hp[a] + omega[a, None] * (
                    dalpha_k[a, None] * Hp[a] + alpha_k[a, None] * dHp[a])
        # seed residual and preconditioned residual
        r = r - alpha * q
        rp, k_in = inner_cg(S, r, inner_tol)
        out.inner_iters += k_in
        rho_next = rp @ r
        beta = rho_next / rho
        p = rp + beta * p
        rho = rho_next
        # frozen shifts keep their pi (their iterates no longer move)
        pi_prev, pi = np.where(a, pi, pi_prev), np.where(a, pi_next, pi)
        if deriv:
            dpi_prev, dpi = np.where(a, dpi, dpi_prev), np.where(a, dpi_next, dpi)
        alpha_prev, beta_prev = alpha, beta
        out.iters = n + 1
        # collinear residual: ||r^k|| = |omega_k| ||r|| / |pi_k|
        res = np.abs(omega) * np.linalg.norm(r) / (np.abs(pi) * bnorm)
        res_final = np.where(active, res, res_final)
        active &= res > tol
        if not active.any():
            break
        if active[s] and (n + 1) not in force_switch:
            continue
        # seed switching: the least-converged active shift becomes the seed
        cand = np.flatnonzero(active & (np.arange(K) != s))
        if cand.size == 0:
            continue
        s_new = int(cand[np.argmax(res[cand])])
        if full:
            c, c_prev = pi[s_new], pi_prev[s_new]
            r = r / c
            rp = rp / c
            rho = rho / c ** 2
            beta_prev = beta_prev * (c_prev / c) ** 2
            alpha_prev = alpha_prev * c_prev / c
            p = rp + beta_prev * P[s_new]
            pi = pi / c
            pi_prev = pi_prev / c_prev
            if deriv:
                dpi = dpi / c
                dpi_prev = dpi_prev / c_prev
            out.switches += 1
        else:
            # collinear restart on the current residual r: every shifted
            # residual is omega_k r / pi_k, so the remaining correction is
            # (omega_k / pi_k) A_k^{-1} r, solved by a fresh process
            if deriv:
                domega = domega / pi - omega * dpi / pi ** 2
                dpi = np.zeros(K, complex)
                dpi_prev = np.zeros(K, complex)
                dHp[:] = 0.0
            omega = omega / pi
            rho = rp @ r
            p = rp.copy()
            alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
            pi = np.ones(K, complex)
            pi_prev = np.ones(K, complex)
            Hp[:] = 0.0
            out.restarts += 1
        s = s_new
        out.seeds.append(s)
    out.res = res_final
    out.converged = out.res <= tol
    return out


def cocg_single(A, S, b, n_steps: int):
    """Plain S-preconditioned COCG on one system A x = b (no shift trick),
    exact inner solves; returns the iterates x_1 ... x_n (brute-force pin)."""
    r = b.astype(np.complex128).copy()
    rp = np.linalg.solve(S, r)
    p = rp.copy()
    rho = rp @ r
    x = np.zeros_like(r)
    xs = []
    for _ in range(n_steps):
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rp = np.linalg.solve(S, r)
        rho_next = rp @ r
        p = rp + (rho_next / rho) * p
        rho = rho_next
        xs.append(x.copy())
    return xs
