"""MI355X-native displacement-based FFT mechanical solver (HIP, gfx950).

The solver itself is the HIP library ``libfmsolve.so`` behind the C ABI of
``include/fmsolve.h``; ``binding`` marshals Python problem descriptions into
it.  Build with ``python -m paper_2607_05929_amd.build``.
"""
from .binding import FmError, LIB_PATH, Plan, batch_solve, lib, solve  # noqa: F401

__all__ = ["FmError", "LIB_PATH", "Plan", "batch_solve", "lib", "solve"]
