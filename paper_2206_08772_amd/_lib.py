"""ctypes view of libotm.so (the C ABI declared in include/otm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotm.so")

OTM_OK, OTM_ERR_ARG, OTM_ERR_CAPACITY, OTM_ERR_LME_NOCONV = 0, -1, -2, -3
OTM_ERR_RM_NOCONV, OTM_ERR_INVERTED, OTM_ERR_NONFINITE, OTM_ERR_HIP = -4, -5, -6, -7
OTM_ERR_SUPPORT, OTM_ERR_SCRATCH = -8, -9
OTM_STATIC_SCRATCH_BYTES = 64 << 20
OTM_FP64, OTM_MIXED, OTM_MIXED_STORAGE = 0, 1, 2
OTM_SCATTER_ATOMIC, OTM_SCATTER_SEGMENTED = 0, 1
OTM_NEOHOOKE, OTM_J2_JC, OTM_J2_LINEAR = 0, 1, 2


class OtmError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().otm_status_string(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg}" if what else msg)


class Params(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("wall_enabled", C.c_int32),
        ("E", C.c_double), ("nu", C.c_double), ("rho0", C.c_double),
        ("A", C.c_double), ("B", C.c_double), ("n", C.c_double), ("C", C.c_double),
        ("m", C.c_double), ("eps_dot0", C.c_double), ("T_r", C.c_double),
        ("T_m", C.c_double), ("Cp", C.c_double), ("chi", C.c_double),
        ("Y0", C.c_double), ("H", C.c_double),
        ("beta", C.c_double), ("r_list", C.c_double), ("cell_size", C.c_double),
        ("lme_tol", C.c_double), ("lme_max_iter", C.c_int32), ("rm_max_iter", C.c_int32),
        ("rm_tol", C.c_double), ("wall_x", C.c_double * 3), ("wall_n", C.c_double * 3),
        ("eps_stab", C.c_double), ("body_force", C.c_double * 3),
        ("fracture", C.c_int32), ("tool_enabled", C.c_int32), ("jc_d", C.c_double * 5),
        ("tool_c", C.c_double * 3), ("tool_v", C.c_double * 3), ("tool_r", C.c_double),
        ("tool_clearance", C.c_double), ("tool_cN", C.c_double), ("tool_cT", C.c_double),
        ("tool_mu", C.c_double), ("kappa", C.c_double), ("insert_dist", C.c_double),
        ("delete_orphans", C.c_int32), ("pad1", C.c_int32),
    ]


class State(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int64), ("n_mp", C.c_int64), ("pair_capacity", C.c_int64),
        ("precision", C.c_int32), ("pad0", C.c_int32),
        ("x", C.c_void_p), ("du", C.c_void_p), ("m", C.c_void_p), ("f", C.c_void_p),
        ("xp", C.c_void_p), ("vol", C.c_void_p), ("mass", C.c_void_p), ("lam", C.c_void_p),
        ("Fd", C.c_void_p), ("bed", C.c_void_p), ("epsbar", C.c_void_p), ("T", C.c_void_p),
        ("sigma", C.c_void_p),
        ("nbr_offsets", C.c_void_p), ("nbr_idx", C.c_void_p), ("N", C.c_void_p),
        ("dN", C.c_void_p), ("xp_prev", C.c_void_p), ("dFm1", C.c_void_p),
        ("failed", C.c_void_p), ("tool_gt", C.c_void_p), ("clock", C.c_void_p),
        ("heat", C.c_void_p), ("qflux", C.c_void_p), ("node_capacity", C.c_int64),
    ]


class Lists(C.Structure):
    """otm_lists: support lists and shape functions of one configuration."""
    _fields_ = [(k, C.c_void_p) for k in ("nbr_offsets", "nbr_idx", "N", "dN")]


class Diag(C.Structure):
    _fields_ = [
        ("flags", C.c_uint32), ("max_support", C.c_int32),
        ("n_lme_noconv", C.c_uint64), ("n_rm_noconv", C.c_uint64),
        ("n_inverted", C.c_uint64), ("n_nonfinite", C.c_uint64),
        ("first_lme_noconv", C.c_uint64), ("first_rm_noconv", C.c_uint64),
        ("first_inverted", C.c_uint64), ("first_nonfinite", C.c_uint64),
        ("pairs_needed", C.c_int64), ("reserved", C.c_int64 * 3),
    ]


class Tape(C.Structure):
    """otm_tape: one stored step of a forward trajectory."""
    _fields_ = [("n_nodes", C.c_int64), ("n_mp", C.c_int64), ("pair_stride", C.c_int64)] + \
        [(k, C.c_void_p) for k in ("x", "du", "m", "f", "xp", "vol", "lam", "Fd", "bed",
                                  "epsbar", "T", "sigma", "nbr_offsets", "nbr_idx", "N", "dN")]


class StateBar(C.Structure):
    """otm_state_bar: adjoint of one step's state."""
    _fields_ = [(k, C.c_void_p) for k in ("x", "du", "vol", "Fd", "bed", "epsbar", "T", "sigma",
                                          "N", "dN")]


_LIB = None

_SIGS = {
    "otm_status_string": (C.c_char_p, [C.c_int32]),
    "otm_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int64]),
    "otm_diag_reset": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "otm_diag_read": (C.c_int32, [C.c_void_p, C.POINTER(Diag), C.c_void_p]),
    "otm_build_neighbors": (C.c_int32, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_double,
                                        C.c_double, C.c_int64, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_int64), C.c_void_p, C.c_size_t,
                                        C.c_void_p]),
    "otm_lme_shape": (C.c_int32, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_int32,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                  C.c_void_p]),
    "otm_init": (C.c_int32, [C.POINTER(State), C.POINTER(Params), C.c_double, C.c_void_p,
                             C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "otm_refresh": (C.c_int32, [C.POINTER(State), C.POINTER(Params), C.c_int32, C.c_int32,
                                C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "otm_step": (C.c_int32, [C.POINTER(State), C.POINTER(Params), C.c_double, C.c_int32,
                             C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "otm_step_into": (C.c_int32, [C.POINTER(State), C.POINTER(Lists), C.POINTER(Params),
                                  C.c_double, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t,
                                  C.c_void_p, C.c_void_p]),
    "otm_erode": (C.c_int32, [C.POINTER(State), C.POINTER(Params), C.c_int32, C.c_void_p,
                              C.c_size_t, C.c_void_p, C.POINTER(C.c_int64),
                              C.POINTER(C.c_int64), C.c_void_p]),
    "otm_step_profiled": (C.c_int32, [C.POINTER(State), C.POINTER(Params), C.c_double,
                                      C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "otm_step_noalloc": (C.c_int32, [C.POINTER(State), C.POINTER(Params), C.c_double,
                                     C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
}

_OPTIONAL = {
    "otm_adjoint_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int64]),
    "otm_init_adjoint": (C.c_int32, [C.c_int64, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "otm_step_adjoint": (C.c_int32, [C.POINTER(Tape), C.POINTER(Tape), C.POINTER(Params),
                                     C.c_double, C.c_void_p, C.POINTER(StateBar),
                                     C.POINTER(StateBar), C.c_void_p, C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.c_void_p]),
}


def lib():
    """The loaded library (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2206_08772_amd.build`")
        # torch first: libotm then binds to the HIP runtime torch loaded (the
        # one its tensors and streams belong to), not to a second copy
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in {**_SIGS, **_OPTIONAL}.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def exported_symbols():
    return sorted(_SIGS) + sorted(_OPTIONAL)


def check(code, what=""):
    if code != OTM_OK:
        raise OtmError(code, what)
    return code
