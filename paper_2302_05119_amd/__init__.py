"""MI355X (gfx950) implementation of CoNCPD-APG / lraCoNCPD-APG.

The compute path is libconcpd.so (hand-written HIP kernels behind the C ABI in
include/concpd.h); this package only marshals arguments to it.
"""
from ._lib import ConcpdError, load  # noqa: F401
from .model import CoupledCP, launch_floor, spectral_norm  # noqa: F401
from .autograd import CoupledCPLoss, coupled_cp_loss  # noqa: F401
