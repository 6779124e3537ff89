"""GMRES-SDR (sketched GMRES with deflated restarting) for MI355X.

The solver is the HIP library ``libsdr.so`` behind the C interface in
``include/sdr.h``; ``paper_2311_14206_amd.sdr`` is its Python binding and
``paper_2311_14206_amd.autograd`` wraps a solve as a differentiable function.
Importing the package loads nothing; the binding loads the library on use.
"""

__all__ = ["SDRSolver", "SDRSolve"]


def __getattr__(name):
    if name == "SDRSolver":
        from .sdr import SDRSolver
        return SDRSolver
    if name == "SDRSolve":
        from .autograd import SDRSolve
        return SDRSolve
    raise AttributeError(name)
