"""FP64 CPU oracle for the RSD-preconditioned Krylov solve.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its Python binding.
"""
from .rsd import Hierarchy, RSDOracle, exact_block_solve  # noqa: F401
from .krylov import fgmres, pcg  # noqa: F401
from . import adjoint  # noqa: F401,E402
