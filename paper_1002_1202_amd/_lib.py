"""ctypes declarations of the gsc C ABI (include/gsc.h).  Loading fails
loudly when the HIP library has not been built: there is no fallback."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsc.so")

GSC_OK, GSC_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "GSC_OK", 1: "GSC_NOT_CONVERGED", -1: "GSC_E_ARG", -2: "GSC_E_NOMEM",
                -3: "GSC_E_DEVICE", -4: "GSC_E_BREAKDOWN", -5: "GSC_E_S_NOT_SPD",
                -6: "GSC_E_NAN", -7: "GSC_E_UNSUPPORTED"}
FP64, MIXED, C64 = 0, 1, 2
CARRY_FULL, CARRY_PROJECTED = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("inner_tol", C.c_double),
                ("inner_max_iter", C.c_int), ("precision", C.c_int), ("carry", C.c_int),
                ("seed_index", C.c_int), ("fuse_steps", C.c_int), ("rhs_tile", C.c_int),
                ("recheck", C.c_int), ("spmm_kernel", C.c_int), ("inner_method", C.c_int),
                ("graph_iters", C.c_int), ("stream_hint", C.c_int), ("cheb_block", C.c_int),
                ("inner_relax", C.c_int), ("batch_streams", C.c_int), ("batch_mem_mb", C.c_int),
                ("row_groups", C.c_int), ("reserved", C.c_int * 1)]


class Stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_longlong), ("switches", C.c_int),
                ("restarts", C.c_int), ("shift_rhs_iters", C.c_longlong), ("seconds", C.c_double),
                ("res_recursive", C.POINTER(C.c_double)), ("res_true", C.POINTER(C.c_double)),
                ("converged", C.POINTER(C.c_ubyte)), ("alg_bytes", C.c_double),
                ("alg_bytes_inner", C.c_double)]


class AsedGeom(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("pos", C.POINTER(C.c_double)),
                ("orb_atom", C.POINTER(C.c_int32)), ("eps", C.POINTER(C.c_double)),
                ("trans", C.POINTER(C.c_double)), ("ang", C.POINTER(C.c_double)),
                ("s0", C.c_double), ("r0", C.c_double), ("lam", C.c_double),
                ("kappa", C.c_double), ("theta", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("pair", C.c_void_p), ("nshift", C.c_int), ("z", C.POINTER(C.c_double)),
                ("nrhs", C.c_int), ("rhs_idx", C.POINTER(C.c_int64)), ("w", C.POINTER(C.c_double)),
                ("g_diag", C.c_void_p), ("q_orb", C.c_void_p), ("e_orb", C.c_void_p),
                ("stats", C.POINTER(Stats))]


# exported symbol -> (restype, argtypes)
class SccOpts(C.Structure):
    _fields_ = [("beta", C.c_double), ("history", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("neutral", C.c_int)]


_VP, _DP, _I64P, _I32P = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
SIGNATURES = {
    "gsc_opts_default": (None, [C.POINTER(Opts)]),
    "gsc_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, _VP]),
    "gsc_set_stream": (C.c_int, [_VP, _VP]),
    "gsc_destroy": (None, [_VP]),
    "gsc_release_cache": (C.c_int, []),
    "gsc_last_error": (C.c_char_p, []),
    "gsc_version": (C.c_char_p, []),
    "gsc_pair_create": (C.c_int, [_VP, C.c_int, C.c_int64, _I64P, _I32P, _VP, _VP, C.c_int,
                                  C.POINTER(C.c_void_p)]),
    "gsc_pair_set_values": (C.c_int, [_VP, _VP, _VP, C.c_int]),
    "gsc_pair_get_values": (C.c_int, [_VP, _VP, _VP, C.c_int]),
    "gsc_pair_info": (C.c_int, [_VP, _I64P, _I64P, C.POINTER(C.c_int)]),
    "gsc_pair_destroy": (None, [_VP]),
    "gsc_ased_build": (C.c_int, [_VP, C.POINTER(AsedGeom), C.c_double, _VP, _DP]),
    "gsc_ased_vjp": (C.c_int, [_VP, C.POINTER(AsedGeom), C.c_double, _VP, _VP, _VP, C.c_int, _DP]),
    "gsc_spmm": (C.c_int, [_VP, _VP, C.c_int, _DP, _VP, _VP, C.c_int]),
    "gsc_spmm_noalloc": (C.c_int, [_VP, _VP, C.c_int, _DP, _VP, _VP]),
    "gsc_solve": (C.c_int, [_VP, _VP, C.c_int, _DP, C.c_int, _I64P, _VP, C.POINTER(Opts), _VP,
                            C.c_int, _I64P, _VP, C.c_int, C.POINTER(Stats)]),
    "gsc_mulliken_band": (C.c_int, [_VP, _VP, C.c_int, _DP, _DP, C.c_int, _I64P, C.POINTER(Opts),
                                    _VP, _VP, _DP, C.c_int, C.POINTER(Stats)]),
    "gsc_band_energy_vjp": (C.c_int, [_VP, _VP, C.c_int, _DP, _DP, C.c_int, _I64P, C.c_double,
                                      C.POINTER(Opts), _VP, _VP, _DP, C.c_int, C.POINTER(Stats)]),
    "gsc_solve_batched": (C.c_int, [_VP, C.c_int, C.POINTER(Problem), C.POINTER(Opts)]),
    "gsc_charge_vjp": (C.c_int, [_VP, _VP, C.c_int, _DP, _DP, C.c_int, _I64P, _DP, C.POINTER(Opts), _VP, _VP,
                                 C.c_int, C.POINTER(Stats)]),
    "gsc_csc_create": (C.c_int, [_VP, _VP, C.POINTER(AsedGeom), _DP, C.POINTER(C.c_void_p)]),
    "gsc_csc_destroy": (None, [_VP]),
    "gsc_csc_potential": (C.c_int, [_VP, _VP, _VP, C.c_int]),
    "gsc_csc_hamiltonian": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int]),
    "gsc_scc_opts_default": (None, [C.POINTER(SccOpts)]),
    "gsc_scc": (C.c_int, [_VP, _VP, _VP, C.c_int, _DP, _DP, _DP, C.POINTER(SccOpts), C.POINTER(Opts), _DP, _DP,
                          _DP, C.POINTER(C.c_int), _DP, _DP]),
    "gsc_lanczos_green": (C.c_int, [_VP, _VP, C.c_int, _DP, C.c_int, _I64P, C.c_int, C.c_double, C.c_int,
                                    C.POINTER(Opts), _VP, _DP, _DP, C.POINTER(C.c_int), C.c_int,
                                    C.POINTER(Stats)]),
    "gsc_profile_enable": (C.c_int, [_VP, C.c_int]),
    "gsc_profile_select": (C.c_int, [_VP, C.c_char_p]),
    "gsc_profile_read": (C.c_int, [_VP, C.c_char_p, _DP, C.POINTER(C.c_longlong), _DP]),
}

KERNELS = ("spmm_seed", "spmm_S", "shift_update", "cg_update", "cg_dir", "update_r", "rho_dot",
           "p_update", "ctrl", "post", "proj_update", "cheb_step", "ring_transpose", "lz_hprod",
           "lz_update", "lz_scale", "cheb_mx", "mx_resid")

_lib = None


def load():
    """Load libgsc.so and declare every C ABI signature.  Raises if the
    library has not been built (run ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, allow_not_converged: bool = True) -> int:
    if status < 0 or (status == GSC_NOT_CONVERGED and not allow_not_converged):
        raise GscError(status, load().gsc_last_error().decode())
    return status
