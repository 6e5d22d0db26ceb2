"""DPDE with energy conservation on MI355X: velocity-Verlet + SER pair-parallel
fluctuation/dissipation (Homman, Maillet, Roussel, Stoltz, arXiv:1507.06643).

The compute lives in libdpde.so (hand-written HIP for gfx950); this package is
its Python binding.  Importing it loads the library and fails loudly when it
has not been built.
"""
# torch first: its HIP runtime is then the one the library binds to (one
# runtime per process, shared streams and device state)
import torch  # noqa: F401

from . import _lib
from ._lib import (DpdeError, EOS_EINSTEIN, EOS_LINEAR, FP32, FP64, MODEL_PROJECTED,
                   MODEL_VECTOR, POT_LJ, POT_SOFT, SCHEME_HYBRID, SCHEME_SEM, SCHEME_SER, THETA_MLP,
                   PAIRS_BOTH_SIDES, PAIRS_ONCE_PER_TILE, THETA_MLP_NEWTON, THETA_NEWTON)

_lib.load()

from .system import (Config, System, debug_rng, tuning_clear, tuning_load,  # noqa: E402
                     tuning_lookup, tuning_save)

__all__ = ["Config", "System", "debug_rng", "DpdeError", "FP32", "FP64", "EOS_LINEAR",
           "MODEL_VECTOR", "MODEL_PROJECTED", "POT_SOFT", "POT_LJ",
           "EOS_EINSTEIN", "THETA_NEWTON", "THETA_MLP", "THETA_MLP_NEWTON", "SCHEME_SER",
           "SCHEME_SEM", "PAIRS_BOTH_SIDES", "PAIRS_ONCE_PER_TILE", "tuning_load",
           "tuning_save", "tuning_clear", "tuning_lookup"]
