"""MI355X-native Monte Carlo closed-loop CSTR (arXiv 2212.02197).

The native library (csrc/, built into libmc_cl.so) holds every step of the
path; `binding` marshals arguments to its C-ABI.  Importing the package does
not load the library; `binding.lib()` does, and fails loudly if it is absent.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
