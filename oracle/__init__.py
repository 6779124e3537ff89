"""Plain FP64 CPU oracle of GMRES-SDR -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package.  The product (the HIP library and its
Python binding) never calls it and shares no code with it.

Contents
--------
``sketch``      the sparse-sign sketching operator S (Section 3, eq. (3.1)):
                an explicit scipy matrix built from a published counter-based
                generator (SplitMix64 output mixer).
``srdct``       the subsampled randomised DCT sketch S = sqrt(N/s) P F E of
                Section 6 (scipy's orthonormal DCT-II).
``gmres_sdr``   GMRES-SDR written from Section 3: truncated Arnoldi,
                sketches, sketched least squares, residual control and the
                harmonic-Ritz compression as separate parts, composed into a
                restart cycle, with the restart and sequence logic of
                Section 3.6, in float64 / complex128, and its right Jacobi
                preconditioned form.
``ilu``         ILU(0) in a greedy multicolour ordering and GMRES-SDR right
                preconditioned with it (Section 6 preconditions by ILU).
"""

from .sketch import sketch_operator, sketch_pattern, splitmix64_mix  # noqa: F401
from .srdct import SRDCT, srdct_rows, srdct_signs  # noqa: F401
from .gmres_sdr import (  # noqa: F401
    Recycle,
    SolveResult,
    sdr_cycle,
    sdr_solve,
    sdr_solve_right_jacobi,
    harmonic_ritz_update,
)
from .ilu import ILU0, greedy_colours, ilu0, multicolour_order, sdr_solve_right_ilu0  # noqa: F401
