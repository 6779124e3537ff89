"""GPU parity of the Givens-rotation residual control (option resid_control=1)
against the oracle's (Sections 4.5 and 5).

The library takes each step's Givens sine as the ratio of consecutive
sketched residuals (the Givens-sine theorem), the oracle rotates the
augmented Hessenberg matrix; both grow the same estimate and refit eps the
same way, so the decision traces, the fitted eps and x must agree.
"""

import numpy as np
import pytest

from oracle import sdr_solve
from workloads import cd2d_upwind, crandn, helmholtz2d, randn, workload

import test_gpu_parity as gp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(A, b, kw, tol, recycle_solver=None, ref_recycle=None, eps0=0.0, **extra):
    h = recycle_solver or gp._solver(A, resid_control=1, givens_eps0=eps0, **kw, **extra)
    x, st = h.solve(gp._dev(b), tol=tol)
    ref = sdr_solve(A.to_scipy(), b, tol=tol, resid_control="givens", givens_eps0=eps0,
                    recycle=ref_recycle, **kw)
    xg = gp._host(x)
    print(f"givens: {st['iters']} steps, {st['res_checks']} checks, eps {st['eps']:.6e} "
          f"(oracle {ref.iters}, {ref.res_checks}, {ref.eps:.6e})", flush=True)
    gp._assert_trace_and_x(xg, st, h.trace(), ref, A=A, b=b, tol=tol)
    assert abs(st["eps"] - ref.eps) <= 1e-8 * max(ref.eps, 1e-300)
    r = b - A.to_scipy() @ xg
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b)
    return h, ref


@pytest.mark.parametrize("dia", [1, 0])
def test_givens_cd2d_64_matches_oracle(dia):
    A, b, p = workload("cd2d_64")
    kw = dict(m=p["m"], k=p["k"], t=p["t"], s=p["s"])
    h, ref = _run(A, b, kw, p["tol"], dia=dia)
    assert ref.refits, "no eps refit happened: the case does not exercise the control"


def test_givens_complex_helmholtz_matches_oracle():
    A = helmholtz2d(32, kappa=8.0)
    _run(A, crandn(A.n, 3), dict(m=40, k=8, t=3, s=96), 1e-9)


def test_givens_initial_eps_and_ragged_sizes():
    A = cd2d_upwind(37)
    _run(A, randn(A.n, 37), dict(m=25, k=5, t=3, s=64), 1e-9, eps0=0.05)


def test_givens_new_rhs_starts_from_the_recycled_block():
    """Second solve with a new right-hand side: the estimate of its first
    cycle is anchored at the sketched residual over span(U) / sqrt(1 - eps)."""
    A = cd2d_upwind(40)
    kw = dict(m=30, k=6, t=2, s=80)
    h, ref = _run(A, randn(A.n, 41), kw, 1e-9)
    _run(A, randn(A.n, 42), kw, 1e-9, recycle_solver=h, ref_recycle=ref.recycle)
