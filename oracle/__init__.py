"""CPU oracle for the interpolated harmonic-mode summation.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  The GPU
library never links or calls it, and it shares no code with the GPU path.
"""
from .oracle import (OracleError, build, load, spline_coefs, swsh, phase,
                     mode_sum, mode_sum_waveform, ORACLE_SO)
from .metrics import mismatch, max_rel_error, inner_flat

__all__ = ["OracleError", "build", "load", "spline_coefs", "swsh", "phase",
           "mode_sum", "mode_sum_waveform", "mismatch", "max_rel_error", "inner_flat",
           "ORACLE_SO"]
