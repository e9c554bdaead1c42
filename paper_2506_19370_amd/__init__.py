"""MI355X-native FC-SDNN per-stage solver (arXiv 2506.19370, Leibovici & Bruno).

The hot path (Euler fluxes, FC-Gram derivative contractions on MFMA, the
smoothness-classifier viscosity, viscous terms, SSPRK stages and overlap
interpolation between curvilinear patches, including C1/C2 corner patches)
runs in hand-written gfx950 HIP kernels behind the C ABI of
``include/fcsdnn.h``; this package is the Python binding.
"""
from ._lib import FcsError, fc_continuation, fc_operator  # noqa: F401
from .api import DerivSweep, SdnnTrainer, Solver, SolverParams, lines_apply, modal_infer, sdnn_infer  # noqa: F401
