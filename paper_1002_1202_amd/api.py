"""Python binding of the gsc C ABI: argument marshalling only.

Host arrays are numpy; device arrays are torch CUDA (HIP) tensors, used as
plain device memory.  Every computation runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


def _ptr(a, ctype=C.c_double):
    """Pointer to a numpy array (host) or a torch tensor (device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data_as(C.POINTER(ctype))
    if not a.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.cast(C.c_void_p(a.data_ptr()), C.POINTER(ctype))


def _vp(a):
    p = _ptr(a)
    return None if p is None else C.cast(p, C.c_void_p)


def _is_device(a) -> bool:
    return a is not None and not isinstance(a, np.ndarray) and getattr(a, "is_cuda", False)


def _complex_view(a):
    """complex128 numpy array -> float64 view (interleaved re, im)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


class Context:
    """One device and one stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = L.load()
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except ImportError:
                stream = None
        h = C.c_void_p()
        L.check(self.lib.gsc_create(C.byref(h), device, C.c_void_p(stream) if stream else None))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.lib.gsc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(ctx: Context, on: bool = True, only: str | None = None):
    """Reset and enable (or disable) live HIP-event timing of every kernel, or
    of the kernel named ``only``.  Algorithmic bytes are counted for all."""
    L.check(ctx.lib.gsc_profile_enable(ctx.h, int(on)))
    if on:
        L.check(ctx.lib.gsc_profile_select(ctx.h, only.encode() if only else None))


def release_cache(ctx: Context) -> None:
    """Hand the library's cached device blocks back to the runtime."""
    L.check(ctx.lib.gsc_release_cache())


def profile_read(ctx: Context) -> dict:
    """{kernel: (total_ms, launches, algorithmic_bytes)} since profile_enable."""
    out = {}
    for name in L.KERNELS:
        ms, n, b = C.c_double(), C.c_longlong(), C.c_double()
        L.check(ctx.lib.gsc_profile_read(ctx.h, name.encode(), C.byref(ms), C.byref(n), C.byref(b)))
        out[name] = (ms.value, n.value, b.value)
    return out


class Pair:
    """Block-sparse H, S pair on the device (copies the pattern)."""

    def __init__(self, ctx: Context, block: int, rowptr, colidx, H=None, S=None):
        self.ctx = ctx
        self.lib = ctx.lib
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        mem = L.MEM_DEVICE if _is_device(H) or _is_device(S) else L.MEM_HOST
        if mem == L.MEM_HOST:
            H = None if H is None else np.ascontiguousarray(H, dtype=np.float64)
            S = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        h = C.c_void_p()
        L.check(self.lib.gsc_pair_create(ctx.h, block, len(self.rowptr) - 1, _ptr(self.rowptr, C.c_int64),
                                         _ptr(self.colidx, C.c_int32), _vp(H), _vp(S), mem, C.byref(h)))
        self.h = h
        n, nnzb, b = C.c_int64(), C.c_int64(), C.c_int()
        L.check(self.lib.gsc_pair_info(h, C.byref(n), C.byref(nnzb), C.byref(b)))
        self.n, self.nnzb, self.block = n.value, nnzb.value, b.value

    def set_values(self, H, S):
        mem = L.MEM_DEVICE if _is_device(H) or _is_device(S) else L.MEM_HOST
        if mem == L.MEM_HOST:
            H = None if H is None else np.ascontiguousarray(H, dtype=np.float64)
            S = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        L.check(self.lib.gsc_pair_set_values(self.h, _vp(H), _vp(S), mem))

    def values(self):
        shape = (self.nnzb, self.block, self.block)
        H = np.empty(shape)
        S = np.empty(shape)
        L.check(self.lib.gsc_pair_get_values(self.h, _vp(H), _vp(S), L.MEM_HOST))
        return H, S

    def close(self):
        if self.h:
            self.lib.gsc_pair_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AsedGeometry:
    """Keeps the host arrays of one geometry alive for the C struct."""

    def __init__(self, system, positions=None):
        p = system.params
        self.pos = np.ascontiguousarray(system.positions if positions is None else positions, dtype=np.float64)
        self.orb_atom = np.ascontiguousarray(system.orb_atom, dtype=np.int32)
        self.eps = np.ascontiguousarray(system.eps, dtype=np.float64)
        self.trans = np.ascontiguousarray(system.trans, dtype=np.float64)
        self.ang = np.ascontiguousarray(system.ang, dtype=np.float64)
        self.struct = L.AsedGeom(self.pos.shape[0], _ptr(self.pos), _ptr(self.orb_atom, C.c_int32),
                                 _ptr(self.eps), _ptr(self.trans), _ptr(self.ang),
                                 p.s0, p.r0, p.lam, p.kappa, p.theta)


def pair_from_system(ctx: Context, system, scale: float = 0.0, positions=None):
    """Pattern of ``system`` plus S, H built on the device by the ASED
    kernels (eq. Hap-1).  Returns (pair, scale c)."""
    pair = Pair(ctx, system.block, system.rowptr, system.colidx)
    c = ased_build(ctx, pair, system, scale, positions)
    return pair, c


def ased_build(ctx: Context, pair: Pair, system, scale: float = 0.0, positions=None) -> float:
    g = AsedGeometry(system, positions)
    out = C.c_double()
    L.check(ctx.lib.gsc_ased_build(ctx.h, C.byref(g.struct), scale, pair.h, C.byref(out)))
    return out.value


def ased_vjp(ctx: Context, pair: Pair, system, scale: float, dH, dS, positions=None) -> np.ndarray:
    g = AsedGeometry(system, positions)
    mem = L.MEM_DEVICE if _is_device(dH) else L.MEM_HOST
    if mem == L.MEM_HOST:
        dH = np.ascontiguousarray(dH, dtype=np.float64)
        dS = np.ascontiguousarray(dS, dtype=np.float64)
    F = np.empty((g.pos.shape[0], 3))
    L.check(ctx.lib.gsc_ased_vjp(ctx.h, C.byref(g.struct), scale, pair.h, _vp(dH), _vp(dS), mem, _ptr(F)))
    return F


def spmm(ctx: Context, pair: Pair, X, alpha_S):
    """Y = alpha_S[c] * S X[:, c] - H X[:, c] for complex X (N, R)."""
    alpha = _complex_view(np.broadcast_to(np.asarray(alpha_S, np.complex128), (X.shape[1],)).copy())
    if _is_device(X):
        import torch
        Y = torch.empty_like(X)
        L.check(ctx.lib.gsc_spmm(ctx.h, pair.h, X.shape[1], _ptr(alpha), _vp(X), _vp(Y), L.MEM_DEVICE))
        return Y
    Xv = np.ascontiguousarray(X, dtype=np.complex128)
    Y = np.empty_like(Xv)
    L.check(ctx.lib.gsc_spmm(ctx.h, pair.h, Xv.shape[1], _ptr(alpha), _vp(Xv.view(np.float64)),
                             _vp(Y.view(np.float64)), L.MEM_HOST))
    return Y


def spmm_noalloc(ctx: Context, pair: Pair, X, alpha_S, Y=None):
    """gsc_spmm_noalloc: Y = alpha_S[c] * S X[:, c] - H X[:, c] for a complex
    (N, R) torch tensor X on the context's device; the library allocates
    nothing (its temporaries live in a fixed per-device scratch array).  Y:
    the caller's output tensor (allocated here when not given)."""
    import torch
    if not (_is_device(X) and X.dtype == torch.complex128 and X.is_contiguous()):
        raise ValueError("X must be a contiguous complex128 device tensor")
    alpha = _complex_view(np.broadcast_to(np.asarray(alpha_S, np.complex128), (X.shape[1],)).copy())
    if Y is None:
        Y = torch.empty_like(X)
    L.check(ctx.lib.gsc_spmm_noalloc(ctx.h, pair.h, X.shape[1], _ptr(alpha), _vp(X), _vp(Y)))
    return Y


def make_opts(tol=1e-10, max_iter=5000, inner_tol=0.0, inner_max_iter=200, precision="fp64",
              carry="full", seed_index=-1, fuse_steps=0, rhs_tile=0, recheck=False,
              spmm_kernel=0, inner_method=0, graph_iters=0, stream_hint=0, cheb_block=0,
              inner_relax=False, batch_streams=0, batch_mem_mb=0, row_groups=0) -> L.Opts:
    """gsc_opts with the library's defaults for every option not given (the
    fields and their meaning are those of gsc_opts in include/gsc.h).
    ``precision``: "fp64"; "mixed" (FP64 seed process, inner S-solve in
    complex64 rounds refined by FP64 residuals: FP64 accuracy); or "c64"
    (complex64 vectors and products throughout, FP64 scalars and dots:
    accuracy limited to about cond(z S - H) times the FP32 epsilon);
    ``carry``: "full" (every x^k) or "projected"; ``inner_relax``: relaxed
    inner tolerance (off by default: the fixed inner tolerance of the
    method)."""
    o = L.Opts()
    L.load().gsc_opts_default(C.byref(o))
    o.tol, o.max_iter, o.inner_tol, o.inner_max_iter = tol, max_iter, inner_tol, inner_max_iter
    o.precision = {"fp64": L.FP64, "mixed": L.MIXED, "c64": L.C64}[precision]
    o.carry = {"full": L.CARRY_FULL, "projected": L.CARRY_PROJECTED}[carry]
    o.seed_index, o.fuse_steps, o.rhs_tile, o.recheck = seed_index, fuse_steps, rhs_tile, int(recheck)
    o.spmm_kernel = spmm_kernel
    o.inner_method = inner_method
    o.graph_iters = graph_iters
    o.stream_hint = stream_hint
    o.cheb_block = cheb_block
    o.inner_relax = int(inner_relax)
    o.batch_streams = batch_streams
    o.batch_mem_mb = batch_mem_mb
    o.row_groups = row_groups
    return o


@dataclass
class SolveResult:
    status: int
    G_cols: object            # (K, R, N) complex or None
    G_proj: object            # (K, R, P) complex or None
    res: np.ndarray           # (K, R) recursive residual estimates
    res_true: np.ndarray | None
    converged: np.ndarray
    outer_iters: int
    inner_iters: int
    switches: int
    restarts: int
    shift_rhs_iters: int
    seconds: float


def _stats(K, R, recheck):
    res = np.zeros((K, R))
    conv = np.zeros((K, R), np.uint8)
    rt = np.zeros((K, R)) if recheck else None
    st = L.Stats()
    st.res_recursive = _ptr(res)
    st.converged = _ptr(conv, C.c_ubyte)
    st.res_true = _ptr(rt) if rt is not None else None
    return st, res, conv, rt


def solve(ctx: Context, pair: Pair, z, rhs=None, B=None, out: str = "host", want_cols: bool = True,
          proj=None, out_cols=None, **opt) -> SolveResult:
    """(z_k S - H) x_k = b_r for all shifts and right-hand sides.

    ``rhs``: orbital indices of unit right-hand sides; ``B``: dense (R, N)
    complex right-hand sides instead.  ``proj``: (R, P) row indices whose
    G values are returned.  ``out``: "host" (numpy) or "device" (torch)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    K = z.shape[0]
    opts = make_opts(**opt)
    rhs_a = None if rhs is None else np.ascontiguousarray(rhs, dtype=np.int64)
    R = len(rhs_a) if rhs_a is not None else B.shape[0]
    N = pair.n
    mem = L.MEM_DEVICE if out == "device" else L.MEM_HOST
    carry_full = opts.carry == L.CARRY_FULL
    Gc = Gp = None
    Bv = None
    if B is not None:
        if mem == L.MEM_DEVICE:
            import torch
            Bv = torch.as_tensor(np.ascontiguousarray(B, np.complex128)).to(f"cuda:{ctx.device}")
        else:
            Bv = _complex_view(B)
    P = 0
    pidx = None
    if proj is not None:
        pidx = np.ascontiguousarray(proj, dtype=np.int64)
        P = pidx.shape[1]
    if mem == L.MEM_DEVICE:
        import torch
        dev = f"cuda:{ctx.device}"
        if out_cols is not None:
            if tuple(out_cols.shape) != (K, R, N) or out_cols.dtype != torch.complex128:
                raise ValueError("out_cols must be a (K, R, N) complex128 device tensor")
            Gc = out_cols
        elif want_cols and carry_full:
            Gc = torch.empty((K, R, N), dtype=torch.complex128, device=dev)
        if P:
            Gp = torch.empty((K, R, P), dtype=torch.complex128, device=dev)
    else:
        if want_cols and carry_full:
            Gc = np.empty((K, R, N), np.complex128)
        if P:
            Gp = np.empty((K, R, P), np.complex128)
    st, res, conv, rt = _stats(K, R, opts.recheck)

    def vp(a):
        if a is None:
            return None
        if isinstance(a, np.ndarray):
            return _vp(a.view(np.float64) if a.dtype == np.complex128 else a)
        return _vp(a)

    status = ctx.lib.gsc_solve(ctx.h, pair.h, K, _ptr(_complex_view(z)), R,
                               _ptr(rhs_a, C.c_int64) if rhs_a is not None else None,
                               vp(Bv), C.byref(opts), vp(Gc), P,
                               _ptr(pidx, C.c_int64) if pidx is not None else None, vp(Gp), mem,
                               C.byref(st))
    L.check(status)
    return SolveResult(status, Gc, Gp, res, rt, conv.astype(bool), st.outer_iters, st.inner_iters,
                       st.switches, st.restarts, st.shift_rhs_iters, st.seconds)


def mulliken_band(ctx: Context, pair: Pair, z, w, orb, **opt):
    """Per-orbital Mulliken charge q, band-energy contribution e and their
    sum (Sec. 2.2).  Returns (q, e, e_band, stats dict)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.float64)
    orb = np.ascontiguousarray(orb, dtype=np.int64)
    K, R = z.shape[0], orb.shape[0]
    opts = make_opts(**opt)
    q = np.empty(R)
    e = np.empty(R)
    eb = C.c_double()
    st, res, conv, _ = _stats(K, R, False)
    status = ctx.lib.gsc_mulliken_band(ctx.h, pair.h, K, _ptr(_complex_view(z)), _ptr(w), R,
                                       _ptr(orb, C.c_int64), C.byref(opts), _vp(q), _vp(e),
                                       C.byref(eb), L.MEM_HOST, C.byref(st))
    L.check(status)
    info = dict(status=status, res=res, converged=conv.astype(bool), outer_iters=st.outer_iters,
                inner_iters=st.inner_iters, switches=st.switches, restarts=st.restarts,
                shift_rhs_iters=st.shift_rhs_iters, seconds=st.seconds)
    return q, e, eb.value, info


def charge_vjp(ctx: Context, pair: Pair, z, w, orbs, qbar, dH=None, dS=None, **opt):
    """Gradients of L = sum_r qbar[r] q_{orbs[r]} (Mulliken charges) on the
    stored entries: dH += dL/dH_bc, dS += dL/dS_bc (zeros when not given;
    numpy or torch device tensors of shape (nnzb, B, B)).  Returns (dH, dS,
    status)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.float64)
    orbs = np.ascontiguousarray(orbs, dtype=np.int64)
    qbar = np.ascontiguousarray(qbar, dtype=np.float64)
    shape = (pair.nnzb, pair.block, pair.block)
    if dH is None:
        dH = np.zeros(shape)
    if dS is None:
        dS = np.zeros(shape)
    mem = L.MEM_DEVICE if _is_device(dH) else L.MEM_HOST
    opts = make_opts(**opt)
    st = L.Stats()
    status = ctx.lib.gsc_charge_vjp(ctx.h, pair.h, z.shape[0], _ptr(_complex_view(z)), _ptr(w), orbs.shape[0],
                                    _ptr(orbs, C.c_int64), _ptr(qbar), C.byref(opts), _vp(dH), _vp(dS), mem,
                                    C.byref(st))
    L.check(status)
    return dH, dS, status


class Csc:
    """Charge-self-consistent term on a pair's pattern (Sec. 2.2, eq.
    Hap-CSC): gamma on the coupled atom pairs for the geometry of
    ``system`` and on-site hardness ``U`` (eV, one per atom)."""

    def __init__(self, ctx: Context, pair: Pair, system, U, positions=None):
        self.ctx = ctx
        self.n_atoms = int(system.n_atoms)
        geom = AsedGeometry(system, positions)
        U = np.ascontiguousarray(U, dtype=np.float64)
        h = C.c_void_p()
        L.check(ctx.lib.gsc_csc_create(ctx.h, pair.h, C.byref(geom.struct), _ptr(U), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.gsc_csc_destroy(self.h)
            self.h = None

    def potential(self, dq):
        """V = gamma dq (host arrays)."""
        dq = np.ascontiguousarray(dq, dtype=np.float64)
        V = np.empty(self.n_atoms)
        L.check(self.ctx.lib.gsc_csc_potential(self.h, _vp(dq), _vp(V), L.MEM_HOST))
        return V

    def hamiltonian(self, pair: Pair, H0, dq):
        """Set the pair's H to H0 + H^CSC(dq); H0 (nnzb, B, B) host or device."""
        mem = L.MEM_DEVICE if _is_device(H0) else L.MEM_HOST
        if mem == L.MEM_HOST:
            H0 = np.ascontiguousarray(H0, dtype=np.float64)
            dq = np.ascontiguousarray(dq, dtype=np.float64)
        L.check(self.ctx.lib.gsc_csc_hamiltonian(self.h, pair.h, _vp(H0), _vp(dq), mem))

    def scc(self, pair: Pair, z, w, valence, dq0=None, beta=0.2, history=4, scc_tol=1e-8, max_iter=100,
            neutral=False, **opt):
        """Self-consistency loop (Anderson mixing) to max |dq_out - dq_in| <=
        scc_tol; ``opt`` are the solver options of each charge evaluation;
        ``neutral``: E_F set each iteration by charge neutrality (``w`` not
        used).  Returns a dict with dq, q_orb, e_band, e_fermi, iterations,
        residual and status; the pair keeps H0 + H^CSC(dq)."""
        z = np.ascontiguousarray(z, dtype=np.complex128)
        w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        valence = np.ascontiguousarray(valence, dtype=np.float64)
        dq = np.zeros(self.n_atoms) if dq0 is None else np.array(dq0, dtype=np.float64)
        q = np.empty(pair.n)
        so = L.SccOpts(beta, history, scc_tol, max_iter, int(neutral))
        opts = make_opts(**opt)
        eb = C.c_double()
        it = C.c_int()
        res = C.c_double()
        ef = C.c_double()
        status = self.ctx.lib.gsc_scc(self.ctx.h, self.h, pair.h, z.shape[0], _ptr(_complex_view(z)),
                                      None if w is None else _ptr(w), _ptr(valence), C.byref(so), C.byref(opts),
                                      _ptr(dq), _ptr(q), C.byref(eb), C.byref(it), C.byref(res), C.byref(ef))
        L.check(status)
        return dict(dq=dq, q_orb=q, e_band=eb.value, e_fermi=ef.value, iterations=it.value, residual=res.value,
                    status=status)


@dataclass
class LanczosResult:
    G_diag: object          # [K][R] complex128 (numpy or torch device tensor)
    a: np.ndarray           # [R][m_max] Lanczos coefficients a_n
    b: np.ndarray           # [R][m_max] b_n (b_0 = 0)
    steps: np.ndarray       # [R] steps taken per right-hand side
    status: int
    outer_iters: int
    inner_iters: int
    shift_rhs_iters: int
    seconds: float


def lanczos_green(ctx: Context, pair: Pair, z, rhs, m_max: int = 2000, tol: float = 1e-10, check_every: int = 16,
                  out: str = "host", **opt) -> LanczosResult:
    """Diagonal Green's-function elements G_jj(z_k), j in rhs, by the
    generalised Lanczos process and its continued fraction (Sec. 3.2).
    ``out``: "host" (numpy) or "device" (torch) for G_diag."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    rhs = np.ascontiguousarray(rhs, dtype=np.int64)
    K, R = z.shape[0], rhs.shape[0]
    opts = make_opts(**opt)
    if out == "device":
        import torch
        G = torch.empty((K, R), dtype=torch.complex128, device=f"cuda:{ctx.device}")
        mem = L.MEM_DEVICE
    else:
        G = np.empty((K, R), dtype=np.complex128)
        mem = L.MEM_HOST
    a = np.zeros((R, m_max))
    b = np.zeros((R, m_max))
    steps = np.zeros(R, dtype=np.int32)
    st = L.Stats()
    status = ctx.lib.gsc_lanczos_green(ctx.h, pair.h, K, _ptr(_complex_view(z)), R, _ptr(rhs, C.c_int64), m_max,
                                       float(tol), check_every, C.byref(opts),
                                       C.cast(C.c_void_p(G.data_ptr()), C.c_void_p) if mem == L.MEM_DEVICE
                                       else _vp(G.view(np.float64)), _ptr(a), _ptr(b), _ptr(steps, C.c_int), mem,
                                       C.byref(st))
    L.check(status)
    return LanczosResult(G, a, b, steps, status, st.outer_iters, st.inner_iters, st.shift_rhs_iters, st.seconds)


def band_energy_vjp(ctx: Context, pair: Pair, z, w, grad_E: float = 1.0, dH=None, dS=None, orbs=None, **opt):
    """Band energy over all orbitals and its gradients on the stored entries:
    dH += grad_E dE/dH_bc, dS += grad_E dE/dS_bc (zeros when not given).
    ``dH``/``dS`` may be numpy (host) or torch device tensors of shape
    (nnzb, B, B).  ``orbs``: the columns c this call covers (default every
    orbital); calls over a partition of the orbitals add up to the full
    gradient, and the returned E_band is the sum of e_c over ``orbs``.
    Returns (dH, dS, E_band, info)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.float64)
    K = z.shape[0]
    if orbs is None:
        norb, optr = pair.n, None
    else:
        orbs = np.ascontiguousarray(orbs, dtype=np.int64)
        norb, optr = orbs.shape[0], _ptr(orbs, C.c_int64)
    opts = make_opts(**opt)
    shape = (pair.nnzb, pair.block, pair.block)
    if dH is None:
        dH = np.zeros(shape)
    if dS is None:
        dS = np.zeros(shape)
    mem = L.MEM_DEVICE if _is_device(dH) else L.MEM_HOST
    if mem == L.MEM_HOST:
        dH = np.ascontiguousarray(dH, dtype=np.float64)
        dS = np.ascontiguousarray(dS, dtype=np.float64)
    eb = C.c_double()
    st, res, conv, _ = _stats(K, norb, False)
    status = ctx.lib.gsc_band_energy_vjp(ctx.h, pair.h, K, _ptr(_complex_view(z)), _ptr(w), norb, optr, grad_E,
                                         C.byref(opts), _vp(dH), _vp(dS), C.byref(eb), mem, C.byref(st))
    L.check(status)
    info = dict(status=status, res=res, converged=conv.astype(bool), outer_iters=st.outer_iters,
                inner_iters=st.inner_iters, restarts=st.restarts, shift_rhs_iters=st.shift_rhs_iters,
                seconds=st.seconds)
    return dH, dS, eb.value, info


def pair_values_device(pair: Pair):
    """Copies of the pair's H, S values as torch device tensors."""
    import torch
    shape = (pair.nnzb, pair.block, pair.block)
    H = torch.empty(shape, dtype=torch.float64, device=f"cuda:{pair.ctx.device}")
    S = torch.empty_like(H)
    L.check(pair.lib.gsc_pair_get_values(pair.h, _vp(H), _vp(S), L.MEM_DEVICE))
    return H, S


def solve_batched(ctx: Context, problems, **opt):
    """Solve many systems together (projected carry).  ``problems``: list of
    dicts with keys pair, z, rhs and optionally w.  Returns a list of dicts
    with G_jj (K, R) complex, q and e (R,) when w was given, and stats."""
    import torch
    opts = make_opts(**opt)
    n = len(problems)
    arr = (L.Problem * n)()
    keep = []
    outs = []
    dev = f"cuda:{ctx.device}"
    for i, pb in enumerate(problems):
        z = np.ascontiguousarray(pb["z"], dtype=np.complex128)
        rhs = np.ascontiguousarray(pb["rhs"], dtype=np.int64)
        K, R = z.shape[0], rhs.shape[0]
        zv = _complex_view(z)
        g = torch.empty((K, R), dtype=torch.complex128, device=dev)
        w = pb.get("w")
        wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        q = torch.empty(R, dtype=torch.float64, device=dev) if w is not None else None
        e = torch.empty(R, dtype=torch.float64, device=dev) if w is not None else None
        st, res, conv, _ = _stats(K, R, False)
        arr[i].pair = pb["pair"].h
        arr[i].nshift = K
        arr[i].z = _ptr(zv)
        arr[i].nrhs = R
        arr[i].rhs_idx = _ptr(rhs, C.c_int64)
        arr[i].w = _ptr(wv) if wv is not None else None
        arr[i].g_diag = _vp(g)
        arr[i].q_orb = _vp(q) if q is not None else None
        arr[i].e_orb = _vp(e) if e is not None else None
        arr[i].stats = C.pointer(st)
        keep.append((zv, rhs, wv, st))
        outs.append(dict(G_jj=g, q=q, e=e, res=res, converged=conv, stats=st))
    status = ctx.lib.gsc_solve_batched(ctx.h, n, arr, C.byref(opts))
    L.check(status)
    for o in outs:
        st = o.pop("stats")
        o.update(status=status, outer_iters=st.outer_iters, inner_iters=st.inner_iters,
                 shift_rhs_iters=st.shift_rhs_iters, seconds=st.seconds,
                 alg_bytes=st.alg_bytes, alg_bytes_inner=st.alg_bytes_inner,
                 converged=o["converged"].astype(bool))
    del keep
    return outs
