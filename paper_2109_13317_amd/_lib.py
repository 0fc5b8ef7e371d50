"""ctypes declarations of the C ABI in include/pffrg.h (libpffrg.so).

Argument marshalling only.  Loading fails loudly when the HIP library has not
been built: there is no CPU fallback for any entry point.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpffrg.so")

P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double

OK, EINVAL, EHIP, ENOMEM, EDIVERGED, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
EULER, RK4, DOPRI54 = 0, 1, 2
VERTEX_MODES = {"auto": -1, "one_launch": 0, "separate": 1, "concurrent": 2}


class Lattice(ctypes.Structure):
    _fields_ = [("n_pairs", I), ("swap", P), ("mult", P), ("rpa_off", P), ("rpa_ka", P),
                ("rpa_kb", P), ("rpa_cnt", P), ("coupling", P), ("n_basis", I),
                ("n_sites_total", I), ("site_pair", P), ("site_pos", P), ("basis_pos", P)]


class Mesh(ctypes.Structure):
    _fields_ = [("n_freq", I), ("omega", P)]


class SpinRot(ctypes.Structure):
    _fields_ = [("n_rot", I), ("rot", P), ("swap_rot", P), ("rpa_rot_a", P), ("rpa_rot_b", P),
                ("site_rot", P)]


class FlowOpts(ctypes.Structure):
    _fields_ = [("scheme", I), ("n_lambda", I), ("lambdas", P), ("lam_start", D),
                ("lam_stop", D), ("rtol", D), ("atol", D), ("h0", D), ("hmin", D),
                ("max_steps", I), ("n_k", I), ("d_k", P), ("d_chi_k", P),
                ("resume", I), ("resume_ladder", I), ("resume_log_lambda", D)]


OBSERVER = ctypes.CFUNCTYPE(ctypes.c_int, D, P, P, P)

# name -> (argtypes); every entry point returns pffrg_status (int)
SIGNATURES = {
    "pffrg_create": [ctypes.POINTER(Lattice), ctypes.POINTER(Mesh), I, P, ctypes.POINTER(P)],
    "pffrg_create_xyz": [ctypes.POINTER(Lattice), P, ctypes.POINTER(Mesh), I, P, ctypes.POINTER(P)],
    "pffrg_create_tri": [ctypes.POINTER(Lattice), P, P, ctypes.POINTER(Mesh), I, P, ctypes.POINTER(P)],
    "pffrg_destroy": [P],
    "pffrg_set_stream": [P, P],
    "pffrg_set_vertex_mode": [P, I],
    "pffrg_state_size": [P, ctypes.POINTER(ctypes.c_size_t)],
    "pffrg_init_state": [P, P],
    "pffrg_rhs": [P, D, P, P],
    "pffrg_sigma_rhs": [P, D, P, P],
    "pffrg_step": [P, I, D, D, P],
    "pffrg_flow": [P, ctypes.POINTER(FlowOpts), P, OBSERVER, P, ctypes.POINTER(I)],
    "pffrg_flow_position": [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I)],
    "pffrg_chi": [P, D, P, P],
    "pffrg_chi_k": [P, P, I, P, P],
    "pffrg_chi_sites": [P, P, P],
    "pffrg_chi_noalloc": [I, P, I, P, D, P, P, P],
    "pffrg_measure_peaks": [P, P],
    "pffrg_set_profiling": [P, I],
    "pffrg_set_profiling_mask": [P, ctypes.c_uint],
    "pffrg_profile_read": [P, I, ctypes.POINTER(D), ctypes.POINTER(I)],
    "pffrg_init_state_from": [P, P, P],
    "pffrg_rhs_vjp": [P, D, P, P, P],
    "pffrg_chi_vjp": [P, D, P, P, P],
    "pffrg_chi_k_vjp": [P, P, I, P, P],
    "pffrg_flow_checkpoints": [P, I, P, P, P],
    "pffrg_flow_vjp": [P, I, P, P, P, P],
    "pffrg_batch_create": [I, ctypes.POINTER(ctypes.POINTER(Lattice)), ctypes.POINTER(Mesh), I, P,
                           ctypes.POINTER(P)],
    "pffrg_batch_destroy": [P],
    "pffrg_batch_state_offsets": [P, ctypes.POINTER(ctypes.c_size_t)],
    "pffrg_batch_init_state": [P, P],
    "pffrg_batch_rhs": [P, D, P, P],
    "pffrg_batch_flow": [P, I, P, P, I, ctypes.POINTER(I)],
    "pffrg_batch_chi": [P, D, P, P],
    "pffrg_batch_chi_k": [P, I, P, I, P, P],
    "pffrg_batch_tune": [P, D, P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)],
    "pffrg_batch_set_launch": [P, I, I, I],
    "pffrg_batch_set_profiling": [P, I],
    "pffrg_batch_profile_read": [P, ctypes.POINTER(D), ctypes.POINTER(I)],
}

K_SIGMA, K_TABLES, K_VERTEX, K_VERTEX_S, K_VERTEX_U, K_VERTEX_T, K_VERTEX_STU = 0, 1, 2, 3, 4, 5, 6

_lib = None


class PffrgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load():
    """The loaded library; raises if libpffrg.so was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_2109_13317_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.pffrg_last_error.restype = ctypes.c_char_p
        lib.pffrg_last_error.argtypes = []
        lib.pffrg_status_string.restype = ctypes.c_char_p
        lib.pffrg_status_string.argtypes = [I]
        _lib = lib
    return _lib


def check(status: int):
    if status != OK:
        lib = load()
        raise PffrgError(status, lib.pffrg_last_error().decode() or
                         lib.pffrg_status_string(status).decode())
    return status
