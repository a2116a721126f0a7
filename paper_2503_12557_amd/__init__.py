"""MI355X (gfx950) library for sampled finite-PEPS amplitudes, local energies,
log-derivatives and the minSR update (arXiv 2503.12557).

The compute path is libpepsmin.so (hand-written HIP kernels behind the
C-ABI of include/pepsmin.h); ``binding`` marshals torch tensors into it.
"""
from .binding import Context, PepsError, load  # noqa: F401
from . import hamiltonians  # noqa: F401
