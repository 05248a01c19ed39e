"""MI355X-native RK3 step of ERF's compressible dynamical core.

The solver is the HIP library ``liberf.so`` behind the C-ABI declared in
``include/erf.h``; ``paper_2412_04395_amd.erf`` is its thin Python binding.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
