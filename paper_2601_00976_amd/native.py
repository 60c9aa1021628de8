"""ctypes binding of ``libnmc.so`` (declared in ``include/nmc.h``).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are passed as torch tensors (their device pointers); torch supplies
device memory and streams.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmc.so")
PROBE_LIB_PATH = os.path.join(HERE, "libnmc_probe.so")

NMC_OK = 0
NMC_E_INVALID_ARG = -1
NMC_E_UNSUPPORTED = -2
NMC_E_HIP = -3
NMC_E_WORKSPACE = -4

STATUS_OK, STATUS_MAX_OUTER, STATUS_MAX_INNER, STATUS_NONFINITE, STATUS_EOS_DOMAIN = 0, 1, 2, 3, 4
NU_E, NU_E_BAR, NU_X = 0, 1, 2
EMAB, ISO, NES, PAIR = 1, 2, 4, 8
ALL_PHYSICS = 15
KERNELS_ON_CHIP, KERNELS_HBM, KERNELS_REGEN, KERNELS_REGISTERS, KERNELS_PAIRED, KERNELS_WAVE = 0, 1, 2, 3, 4, 5
SPACING_LOG, SPACING_ZOOM = 0, 1

EXPORTED = (
    "nmc_model_desc_default", "nmc_solver_params_default", "nmc_grid_create", "nmc_grid_query",
    "nmc_grid_destroy", "nmc_model_create", "nmc_model_destroy", "nmc_workspace_bytes", "nmc_kernel_store_bytes",
    "nmc_solve_batch", "nmc_solve_batch_noalloc", "nmc_solve_batch_v", "nmc_solve_batch_adjoint",
    "nmc_c2p_params_default", "nmc_primitive_recovery", "nmc_pdars_workspace_bytes", "nmc_pdars_step_v",
    "nmc_init_state", "nmc_error_string",
    "nmc_last_error",
)


class NmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nmc error {code}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("nodes_per_elem", C.c_int), ("eps_lo", C.c_double),
                ("eps_hi", C.c_double), ("spacing", C.c_int), ("zoom", C.c_double)]


class ModelDesc(C.Structure):
    _fields_ = [("n_species", C.c_int), ("species", C.c_int * 3), ("flags", C.c_uint),
                ("chi_ref", C.c_double), ("eps_ref", C.c_double), ("chi_power", C.c_double),
                ("sigma_ratio", C.c_double), ("eos_a", C.c_double), ("eos_b", C.c_double),
                ("mu_a", C.c_double), ("mu_ye0", C.c_double), ("mu_b", C.c_double), ("mu_t0", C.c_double),
                ("hc_mev_cm", C.c_double), ("m_u_g", C.c_double), ("rho11_min", C.c_double),
                ("phi1_nes", C.c_double), ("phi1_pair", C.c_double),
                ("fd_projection", C.c_int), ("deq_min", C.c_double), ("deq_max", C.c_double)]


class SolverParams(C.Structure):
    _fields_ = [("tol_inner", C.c_double), ("tol_outer", C.c_double), ("m_inner", C.c_int),
                ("m_outer", C.c_int), ("max_inner", C.c_int), ("max_outer", C.c_int),
                ("fixed_matter", C.c_int)]


class BatchIn(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("D0", "I0", "rho11", "ye0", "e0", "chi0", "T_fixed", "mu_fixed", "theta")]


class BatchOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("D", "I", "ye", "e", "T", "n_outer", "n_inner", "status")]


class BatchVIn(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("D0", "I0", "rho11", "ye0", "ef0", "v0", "chi0", "theta")]


class BatchVOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("D", "I", "ye", "ef", "v", "T", "n_outer", "n_inner", "status")]


class C2pParams(C.Structure):
    _fields_ = [("mem", C.c_int), ("tol", C.c_double), ("max_it", C.c_int)]


class Launch(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int), ("chunk", C.c_int), ("persistent", C.c_int), ("kernel_store", C.c_int)]


_lib = None


def lib():
    """Load libnmc.so (built in-tree by ``paper_2601_00976_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_00976_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.nmc_model_desc_default.argtypes = [C.POINTER(ModelDesc)]
        L.nmc_model_desc_default.restype = None
        L.nmc_solver_params_default.argtypes = [C.POINTER(SolverParams)]
        L.nmc_solver_params_default.restype = None
        L.nmc_grid_create.argtypes = [C.POINTER(GridDesc), C.POINTER(vp)]
        L.nmc_grid_query.argtypes = [vp, C.POINTER(C.c_int), vp, vp, vp]
        L.nmc_grid_destroy.argtypes = [vp]
        L.nmc_model_create.argtypes = [vp, C.POINTER(ModelDesc), C.POINTER(vp)]
        L.nmc_model_destroy.argtypes = [vp]
        L.nmc_workspace_bytes.argtypes = [vp, C.c_int64]
        L.nmc_workspace_bytes.restype = C.c_size_t
        L.nmc_kernel_store_bytes.argtypes = [vp, C.c_int64]
        L.nmc_kernel_store_bytes.restype = C.c_size_t
        L.nmc_solve_batch.argtypes = [vp, C.POINTER(SolverParams), C.c_int64, C.c_double, C.POINTER(BatchIn),
                                      C.POINTER(BatchOut), vp, C.c_size_t, C.POINTER(Launch), vp]
        L.nmc_solve_batch_noalloc.argtypes = [vp, C.POINTER(SolverParams), C.c_int64, C.c_double, C.POINTER(BatchIn),
                                              C.POINTER(BatchOut), C.POINTER(Launch), vp]
        L.nmc_solve_batch_v.argtypes = [vp, C.POINTER(SolverParams), C.c_int64, C.c_double, C.POINTER(BatchVIn),
                                        C.POINTER(BatchVOut), vp, C.c_size_t, C.POINTER(Launch), vp]
        L.nmc_c2p_params_default.argtypes = [C.POINTER(C2pParams)]
        L.nmc_c2p_params_default.restype = None
        L.nmc_primitive_recovery.argtypes = [vp, C.POINTER(C2pParams), C.c_int64, vp, vp, vp, vp, vp, vp, vp]
        L.nmc_pdars_workspace_bytes.argtypes = [vp, C.c_int64]
        L.nmc_pdars_workspace_bytes.restype = C.c_size_t
        L.nmc_pdars_step_v.argtypes = [vp, C.POINTER(SolverParams), C.POINTER(C2pParams), C.c_int64, C.c_double,
                                       C.POINTER(BatchVIn), C.POINTER(BatchVOut), vp, C.c_size_t, C.POINTER(Launch),
                                       vp]
        L.nmc_solve_batch_adjoint.argtypes = [vp, C.POINTER(SolverParams), C.c_int64, C.c_double, C.POINTER(BatchIn),
                                              C.POINTER(BatchOut), vp, vp, vp, vp, C.c_size_t, vp]
        L.nmc_init_state.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                     vp, vp, vp, vp]
        L.nmc_error_string.argtypes = [C.c_int]
        L.nmc_error_string.restype = C.c_char_p
        L.nmc_last_error.argtypes = []
        L.nmc_last_error.restype = C.c_char_p
        for f in ("nmc_grid_create", "nmc_grid_query", "nmc_grid_destroy", "nmc_model_create", "nmc_model_destroy",
                  "nmc_solve_batch", "nmc_solve_batch_noalloc", "nmc_solve_batch_v", "nmc_solve_batch_adjoint", "nmc_init_state",
                  "nmc_primitive_recovery", "nmc_pdars_step_v"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int):
    if rc != NMC_OK:
        raise NmcError(rc, lib().nmc_last_error().decode())
    return rc


def ptr(t):
    """Device (or host) pointer of a tensor, None for None."""
    return None if t is None else C.c_void_p(t.data_ptr())
