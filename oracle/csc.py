"""Charge-self-consistent (CSC) term and the self-consistency loop.

TEST INFRASTRUCTURE ONLY (see the package header).  FP64, plain code written
from Sec. 2.2 (eq. Hap-CSC):

    H^CSC_{ia,jb} = 1/2 S_{ia,jb} sum_k (gamma_ik + gamma_jk) dq_k
                  = 1/2 S_{ia,jb} (V_i + V_j),   V = gamma dq,

with dq_k the deviation of the Mulliken charge of atom k.  The section gives
neither gamma nor the loop; readings used here:
  * gamma_ik (eV) on the atom pairs that the pair's block pattern couples
    (every atom of block row I with every atom of block column J, with that
    block's lattice translation): gamma_ii = U_i on the atom itself, else the
    Klopman-Ohno form e^2 / sqrt(r^2 + a^2), a = e^2 (1/U_i + 1/U_k) / 2,
    e^2 = 14.399645 eV A;
  * dq_k = Q_k - Z_k with Q_k the Mulliken electron count of atom k (sum of
    the orbital charges q_a over its orbitals) and Z_k its valence;
  * loop: dq_in = 0; H = H0 + H^CSC(dq_in); Mulliken charges with the given
    shifts and weights (or, with the neutrality rule, with the Fermi level
    E_F set each iteration so that the charges sum to the valence count:
    trapezoid weights over Re z truncated at E_F, the integrand linear
    between samples, E_F by bisection; no extra solve); dq_out; stop when
    max |dq_out - dq_in| <= tol, else
    the next input by Anderson mixing of the last m residuals f = dq_out -
    dq_in (plain linear mixing dq_in += beta f when m = 0): with the
    differences dF, dX of consecutive residuals and inputs, g minimises
    |f - dF g| and dq_in <- dq_in + beta f - (dX + beta dF) g.
"""
from __future__ import annotations

import numpy as np

from . import green

E2 = 14.399645  # e^2 / (4 pi eps0) in eV * Angstrom


def atom_pairs(system):
    """(a, k, displacement) for every atom pair the block pattern couples."""
    B = system.block
    rows = system.block_rows()
    out = []
    for b in range(system.nnzb):
        I, J = int(rows[b]), int(system.colidx[b])
        atoms_i = sorted(set(int(x) for x in system.orb_atom[I * B:(I + 1) * B]))
        atoms_j = sorted(set(int(x) for x in system.orb_atom[J * B:(J + 1) * B]))
        for a in atoms_i:
            for k in atoms_j:
                d = system.positions[k] + system.trans[b] - system.positions[a]
                out.append((a, k, d))
    return out


def gamma_matrix(system, U, positions=None):
    """Dense gamma (n_atoms x n_atoms), summed over the coupled pairs."""
    if positions is not None:
        system = _with_positions(system, positions)
    n = system.n_atoms
    G = np.zeros((n, n))
    for a, k, d in atom_pairs(system):
        r = float(np.sqrt(d @ d))
        if a == k and r == 0.0:
            G[a, k] += U[a]
        else:
            h = 0.5 * E2 * (1.0 / U[a] + 1.0 / U[k])
            G[a, k] += E2 / np.sqrt(r * r + h * h)
    return G


def _with_positions(system, positions):
    import dataclasses
    return dataclasses.replace(system, positions=np.asarray(positions, dtype=np.float64))


def hamiltonian(S, H0, V, orb_atom):
    """H0 + H^CSC for the atom potentials V (dense; zero wherever S is)."""
    Vo = np.asarray(V)[np.asarray(orb_atom)]
    return H0 + 0.5 * S * (Vo[:, None] + Vo[None, :])


def atom_charges(q_orb, orb_atom, n_atoms):
    Q = np.zeros(n_atoms)
    np.add.at(Q, np.asarray(orb_atom), q_orb)
    return Q


def charge_response(system, S, H0, gamma, z, w, dq_in):
    """dq_out and the band energy for the input charges dq_in (all orbitals)."""
    H = hamiltonian(S, H0, gamma @ dq_in, system.orb_atom)
    orbs = np.arange(system.n)
    X = green.solve_dense(H, S, z, orbs)
    q, e, eb = green.mulliken_band(S, X, z, w, orbs)
    Q = atom_charges(q, system.orb_atom, system.n_atoms)
    return Q - system.valence, q, eb


def truncated_weights(E, e_fermi):
    """Weights w_k with sum_k w_k f(E_k) = integral of f from E_0 to e_fermi
    for f linear between the samples E (ascending): full trapezoid intervals
    below the interval holding e_fermi, and the part of that interval up to
    e_fermi integrated under the interpolating line."""
    E = np.asarray(E, dtype=np.float64)
    K = E.shape[0]
    w = np.zeros(K)
    if e_fermi <= E[0]:
        return w
    for j in range(K - 1):
        h = E[j + 1] - E[j]
        if e_fermi >= E[j + 1]:
            w[j] += 0.5 * h
            w[j + 1] += 0.5 * h
            continue
        d = e_fermi - E[j]
        # integral over [E_j, E_j + d] of f_j + (f_{j+1} - f_j) s / h
        w[j] += d - 0.5 * d * d / h
        w[j + 1] += 0.5 * d * d / h
        break
    return w


def electron_count(E, t, e_fermi):
    """Electrons below e_fermi from t_k = sum_a Im (S G(z_k))_aa:
    N = -(2/pi) sum_k w_k(e_fermi) t_k (spin 2)."""
    return float(-(2.0 / np.pi) * truncated_weights(E, e_fermi) @ np.asarray(t))


def fermi_level(E, t, n_electrons, tol=1e-13):
    """E_F with electron_count(E_F) = n_electrons, by bisection on
    [E_0, E_{K-1}] (the count grows with E_F where -Im Tr(S G) > 0)."""
    lo, hi = float(E[0]), float(E[-1])
    if electron_count(E, t, hi) < n_electrons:
        raise ValueError("the shift grid does not hold the electrons")
    while hi - lo > tol * max(1.0, abs(lo) + abs(hi)):
        mid = 0.5 * (lo + hi)
        if electron_count(E, t, mid) < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def charge_response_neutral(system, S, H0, gamma, z, dq_in):
    """dq_out, q, the band energy and E_F for input charges dq_in, with E_F
    chosen so that the Mulliken charges sum to the valence count."""
    H = hamiltonian(S, H0, gamma @ dq_in, system.orb_atom)
    orbs = np.arange(system.n)
    X = green.solve_dense(H, S, z, orbs)
    sg = np.einsum("ij,kji->ki", S, X)                   # (S G_k)_aa, (K, N)
    E = np.asarray(z).real
    ef = fermi_level(E, sg.imag.sum(axis=1), float(np.sum(system.valence)))
    w = truncated_weights(E, ef)
    q, e, eb = green.mulliken_band(S, X, z, w, orbs)
    Q = atom_charges(q, system.orb_atom, system.n_atoms)
    return Q - system.valence, q, eb, ef


def anderson_step(x, f, X_hist, F_hist, beta):
    """Next input from the current input x, residual f and the previous
    (input, residual) pairs (oldest first)."""
    if not X_hist:
        return x + beta * f
    dX = np.stack([x - xh for xh in X_hist], axis=1)
    dF = np.stack([f - fh for fh in F_hist], axis=1)
    g = np.linalg.lstsq(dF, f, rcond=None)[0]
    return x + beta * f - (dX + beta * dF) @ g


def scc(system, S, H0, gamma, z, w, beta=0.3, tol=1e-8, max_iter=100, dq0=None, history=4, neutral=False):
    """Self-consistency loop with Anderson mixing over `history` previous
    iterates.  Returns (dq, q_orb, e_band, iterations, final residual); dq is
    the last input charge vector.  neutral=True: the weights w are not used,
    E_F is set each iteration by charge neutrality (charge_response_neutral)
    and the last E_F is returned as a sixth value."""
    dq_in = np.zeros(system.n_atoms) if dq0 is None else np.array(dq0, dtype=np.float64)
    X_hist, F_hist = [], []
    res = np.inf
    it = 0
    q = eb = None
    ef = None
    for it in range(1, max_iter + 1):
        if neutral:
            dq_out, q, eb, ef = charge_response_neutral(system, S, H0, gamma, z, dq_in)
        else:
            dq_out, q, eb = charge_response(system, S, H0, gamma, z, w, dq_in)
        f = dq_out - dq_in
        res = float(np.abs(f).max())
        if res <= tol:
            break
        nxt = anderson_step(dq_in, f, X_hist[-history:] if history else [], F_hist[-history:] if history else [],
                            beta)
        X_hist.append(dq_in)
        F_hist.append(f)
        dq_in = nxt
    if neutral:
        return dq_in, q, eb, it, res, ef
    return dq_in, q, eb, it, res
