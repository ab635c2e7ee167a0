"""MI355X (gfx950) S_N upwind-DG transport with ROM-enhanced synthetic acceleration.

The numerical work runs in librte.so (hand-written HIP kernels); ``rte`` is its ctypes binding.
"""
from . import rte  # noqa: F401  (raises ImportError if librte.so has not been built)
