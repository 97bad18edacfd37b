"""MI355X-native differentiable weakly compressible SPH hot path.

The compute path is the HIP library ``libsph.so`` (built from ``csrc/``) behind the
C ABI declared in ``include/sph.h``; ``lib`` is its thin ctypes binding.  Importing
this package loads nothing: the library is opened on first use and a missing
library raises instead of falling back to any other implementation.
"""
__all__ = ["inputs"]
