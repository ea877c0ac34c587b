"""ctypes binding of libgbmc.so (declared in include/gbmc.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgbmc.so")

GBMC_OK = 0
GBMC_ERR_INVALID = -1
GBMC_ERR_HIP = -2
GBMC_ERR_OVERFLOW = -3
GBMC_ERR_UNSUPPORTED = -4
GBMC_FP32_FIXED = 0
GBMC_FP64 = 1
KERNEL_NAMES = ("radii_pairs", "energy_pairs", "chain_pairs", "site_rows", "site_dE", "mc_step",
                "force_pairs", "evaluate_pairs")

_STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "HIP", -3: "OVERFLOW", -4: "UNSUPPORTED"}


class GbmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gbmc status {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class gbmc_gb_params(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("alpha", "beta", "gamma", "offset", "eps_in", "eps_out", "coulomb_k", "kappa",
                 "rgbmax", "cutoff")]


class gbmc_atoms(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "y", "z", "q", "rho", "screen")]


N_PASSES = 3          # descreening, energy/forces, Born chain
PASS_NAMES = ("radii", "energy", "chain")


class gbmc_tuning(C.Structure):
    _fields_ = [("j_blocks_per_item", C.c_int32 * N_PASSES), ("waves_per_group", C.c_int32 * N_PASSES)]


_I32P = C.POINTER(C.c_int32)
_VP = C.c_void_p
_D = C.c_double
_I32 = C.c_int32

# name -> (restype, argtypes); keep in the order of include/gbmc.h
SIGNATURES = {
    "gbmc_version": (_I32, []),
    "gbmc_last_error": (C.c_char_p, []),
    "gbmc_params_validate": (_I32, [C.POINTER(gbmc_gb_params)]),
    "gbmc_schedule_build": (_I32, [_I32, _I32P, _I32, _I32, _I32P, _I32P]),
    "gbmc_queue_schedule": (_I32, [_I32, _I32P, _I32, C.POINTER(gbmc_tuning), _I32P, _I32P, _I32P,
                                   _I32P]),
    "gbmc_plan_create": (_I32, [C.POINTER(_VP), _I32, _I32P, _I32, C.POINTER(gbmc_tuning)]),
    "gbmc_plan_destroy": (None, [_VP]),
    "gbmc_plan_set_order": (_I32, [_VP, _I32P]),
    "gbmc_spatial_order": (_I32, [_I32, _I32P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), _I32P]),
    "gbmc_block_order": (_I32, [_I32, _I32P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double), _I32P]),
    "gbmc_plan_workspace_bytes": (C.c_size_t, [_VP]),
    "gb_radii": (_I32, [_VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP, _VP, _VP]),
    "gb_energy_forces": (_I32, [_VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP, _VP,
                                _VP, _VP, _VP, _VP, _VP]),
    "gb_evaluate": (_I32, [_VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP, _VP, _VP,
                           _VP, _VP, _VP, _VP, _VP]),
    "gb_evaluate_fork": (_I32, [_VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP, _VP,
                                _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "gb_evaluate_static": (_I32, [_VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP,
                                  _VP, _VP, _VP, _VP, _VP, _VP]),
    "gb_plain_workspace_bytes": (C.c_size_t, [_I32]),
    "gb_plain_fp64": (_I32, [_I32, _I32P, _VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP,
                             _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "gbmc_sites_validate": (_I32, [_I32, _I32P, _I32, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P,
                                   _I32P]),
    "gbmc_sites_create": (_I32, [_VP, C.POINTER(_VP), _I32, _I32P, _I32P, _I32P, _I32P, _I32P,
                                 _I32P, C.POINTER(C.c_double), C.POINTER(C.c_double), _I32P]),
    "gbmc_sites_destroy": (None, [_VP]),
    "gbmc_sites_n_candidates": (_I32, [_VP]),
    "gbmc_sites_workspace_bytes": (C.c_size_t, [_VP]),
    "mc_state_dE": (_I32, [_VP, _VP, C.POINTER(gbmc_atoms), C.POINTER(gbmc_gb_params), _VP, _VP,
                           _VP, _VP, _VP, _D, _VP, _VP, _VP]),
    "mc_step": (_I32, [_VP, _VP, C.POINTER(gbmc_atoms), _VP, C.POINTER(gbmc_gb_params), _VP, _VP,
                       _VP, _VP, _VP, _D, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "mc_sweep": (_I32, [_VP, _VP, C.POINTER(gbmc_atoms), _VP, C.POINTER(gbmc_gb_params), _VP, _VP,
                        _VP, _VP, _VP, _D, _I32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "md_langevin_step": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _D, _D, _D, _D, _VP]),
    "remd_exchange": (_I32, [_I32, _VP, _VP, _VP, _D, _I32, _I32, _VP, _VP, _VP, _VP]),
    "gbmc_plan_set_single_launch": (_I32, [_VP, _I32, _I32]),
    "gbmc_plan_set_timing": (_I32, [_VP, _I32]),
    "gbmc_plan_kernel_ms": (_I32, [_VP, C.POINTER(C.c_float)]),
    "gbmc_check_overflow": (_I32, [_VP, _VP, _VP, _I32P]),
}

_lib = None


def load():
    """Load libgbmc.so (raises if it is missing or incomplete)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_1803_09652_amd.build` "
                "(there is no non-HIP fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != GBMC_OK:
        msg = load().gbmc_last_error()
        raise GbmcError(status, msg.decode() if msg else "")
