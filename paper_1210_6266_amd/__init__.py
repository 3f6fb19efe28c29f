"""MI355X-native Recursive Schur Decomposition preconditioned Krylov solver.

The method runs in the HIP library librsd.so (C ABI: include/rsd.h); this
package holds its sources (csrc/), the build script and the ctypes binding.
"""
from .rsd import (RSD, FEMap, RSDError, rsd_analyze, rsd_apply, rsd_destroy,  # noqa: F401
                  rsd_fe_assemble, rsd_fe_grad, rsd_get_stats, rsd_last_error,
                  rsd_options_default, rsd_setup, rsd_solve, rsd_spmv, rsd_update_values)
