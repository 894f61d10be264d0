"""MI355X (gfx950) implementation of the spectral Kohn-Sham H*X hot path and
Chebyshev-filtered subspace iteration (libces.so + a thin ctypes binding)."""
from . import ces  # noqa: F401
