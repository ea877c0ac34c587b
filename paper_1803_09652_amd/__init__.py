"""MI355X-native GB-OBC electrostatics with constant-pH / constant-redox Monte
Carlo and E-REMD exchange (after arXiv:1803.09652).

The compute path is libgbmc.so (HIP kernels for gfx950 behind the C ABI in
include/gbmc.h); this package is its Python binding.
"""
from ._lib import GbmcError, load  # noqa: F401
from .api import (  # noqa: F401
    IGB2, IGB5, KIND_PROT, KIND_REDOX, Atoms, GBEnergy, GBParams, Plan, Sites, block_order,
    check_overflow, energy_forces, evaluate, evaluate_static, md_step, mc_state_dE, mc_step,
    mc_sweep, plain_fp64, radii, remd_exchange, spatial_order,
)

__all__ = ["GbmcError", "load", "IGB2", "IGB5", "KIND_PROT", "KIND_REDOX", "Atoms", "GBEnergy",
           "GBParams", "Plan", "Sites", "block_order", "check_overflow", "energy_forces",
           "evaluate", "evaluate_static", "mc_state_dE", "mc_step", "mc_sweep", "md_step",
           "plain_fp64", "radii", "remd_exchange", "spatial_order"]
