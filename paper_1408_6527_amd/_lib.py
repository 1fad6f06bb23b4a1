"""ctypes binding of libpfmm.so (declarations in include/pfmm.h).

PyTorch is imported first so that its HIP runtime is the one the library binds to (both carry the
SONAME libamdhip64.so.7; the dynamic loader then reuses the copy already in the process).
There is no fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load PyTorch's HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfmm.so")

PFMM_FP64 = 0
PFMM_MIXED = 1
PFMM_WANT_FORCES = 1 << 0
PFMM_WANT_POTENTIALS = 1 << 1
PFMM_SAVE_FOR_BACKWARD = 1 << 2
PFMM_WARM_START = 1 << 3
PFMM_TIMING = 1 << 4

STATUS = {
    0: "PFMM_OK",
    1: "PFMM_ERR_INVALID_ARG",
    2: "PFMM_ERR_NONFINITE",
    3: "PFMM_ERR_COINCIDENT",
    4: "PFMM_ERR_NOT_CONVERGED",
    5: "PFMM_ERR_NOT_SPD",
    6: "PFMM_ERR_OOM",
    7: "PFMM_ERR_HIP",
    8: "PFMM_ERR_NO_STATE",
}


class Config(ctypes.Structure):
    _fields_ = [
        ("order_p", ctypes.c_int),
        ("ws", ctypes.c_int),
        ("leaf_width", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("scf_tol", ctypes.c_double),
        ("scf_max_iter", ctypes.c_int),
        ("graph_iters", ctypes.c_int),
        ("thole_a", ctypes.c_double),
        ("coulomb_k", ctypes.c_double),
        ("flags", ctypes.c_uint),
        ("m2l_order_slack", ctypes.c_int),
        ("precond_cutoff", ctypes.c_double),
        ("precond_iters", ctypes.c_int),
        ("scf_relax", ctypes.c_double),
        ("dipole_pair_dl", ctypes.c_double),
        ("dipole_tree", ctypes.c_int),
        ("mac_theta", ctypes.c_double),
        ("mac_ndirect", ctypes.c_int),
        ("mac_leaf_direct", ctypes.c_int),
        ("adaptive_leaf_max", ctypes.c_int),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("U_total", ctypes.c_double),
        ("U_qq", ctypes.c_double),
        ("U_pol", ctypes.c_double),
        ("iters", ctypes.c_int),
        ("residual", ctypes.c_double),
        ("residual_max_debye", ctypes.c_double),
        ("levels", ctypes.c_int),
        ("leaf_width", ctypes.c_double),
        ("n_leaves", ctypes.c_int64),
        ("n_cells", ctypes.c_int64),
        ("n_m2l", ctypes.c_int64),
        ("n_p2p", ctypes.c_int64),
        ("m2l_flops", ctypes.c_int64),
        ("n_evals", ctypes.c_int),
        ("t_phase_ms", ctypes.c_double * 8),
        ("t_kernel_ms", ctypes.c_double * 8),
        ("kernel_launches", ctypes.c_int * 8),
        ("m2l_flops_total", ctypes.c_int64),
        ("m2l_order_cap_min", ctypes.c_int),
        ("scf_restarts", ctypes.c_int),
        ("solve_id", ctypes.c_int64),
        ("t_m2l_split_ms", ctypes.c_double * 2),
        ("m2l_split_launches", ctypes.c_int * 2),
        ("m2l_split_flops", ctypes.c_int64 * 2),
        ("n_sites", ctypes.c_int64),
    ]

KERNEL_CLASSES = ["p2m", "m2m", "m2l", "l2l", "l2p", "p2p_scf", "p2p_full", "solver"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1408_6527_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pfmm_config_default.argtypes = [ctypes.POINTER(Config)]
    lib.pfmm_config_default.restype = None
    lib.pfmm_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp)]
    lib.pfmm_create.restype = ctypes.c_int
    lib.pfmm_destroy.argtypes = [vp]
    lib.pfmm_destroy.restype = None
    lib.pfmm_solve.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Result), vp]
    lib.pfmm_solve.restype = ctypes.c_int
    lib.pfmm_backward.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp]
    lib.pfmm_backward.restype = ctypes.c_int
    lib.pfmm_solve_qe.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Result), vp]
    lib.pfmm_solve_qe.restype = ctypes.c_int
    lib.pfmm_backward_qe.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp, vp, vp, vp, vp]
    lib.pfmm_backward_qe.restype = ctypes.c_int
    lib.pfmm_backward_mu.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.pfmm_backward_mu.restype = ctypes.c_int
    lib.pfmm_set_exclusions.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.pfmm_set_exclusions.restype = ctypes.c_int
    lib.pfmm_field.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pfmm_field.restype = ctypes.c_int
    lib.pfmm_status_string.argtypes = [ctypes.c_int]
    lib.pfmm_status_string.restype = ctypes.c_char_p
    lib.pfmm_last_error.argtypes = [vp]
    lib.pfmm_last_error.restype = ctypes.c_char_p
    lib.pfmm_version.argtypes = []
    lib.pfmm_version.restype = ctypes.c_char_p
    del dp
    return lib


lib = _load()
