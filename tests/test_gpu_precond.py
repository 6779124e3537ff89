"""GPU parity of right Jacobi preconditioning (option "precond") against the oracle.

The library folds D^-1 = diag(A)^-1 into the stored values and solves
(A D^-1) u = b with x = D^-1 u; the oracle's ``sdr_solve_right_jacobi`` does
the same from its definition.  Inputs are convection-diffusion and Helmholtz
operators with columns scaled by 10^U(-3, 3): a badly scaled unknown per
column, which the unpreconditioned solve handles poorly.
"""

import numpy as np
import pytest

from oracle import sdr_solve, sdr_solve_right_jacobi
from workloads import cd2d_upwind, column_scaled, crandn, helmholtz2d, log_uniform, randn

import test_gpu_parity as gp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KW = dict(m=30, k=6, t=2, s=80)


def _check_against_oracle(A, b, tol, x0=None, extra=None):
    h = gp._solver(A, precond=1, **KW, **(extra or {}))
    x, st = h.solve(gp._dev(b), x=None if x0 is None else gp._dev(x0), tol=tol)
    ref = sdr_solve_right_jacobi(A.to_scipy(), b, x0=x0, tol=tol, **KW)
    gp._assert_trace_and_x(gp._host(x), st, h.trace(), ref, A=A, b=b, tol=tol)
    r = b - A.to_scipy() @ gp._host(x)
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b)
    return h, st, ref


@pytest.mark.parametrize("dia", [1, 0])
def test_jacobi_cd2d_matches_oracle(dia):
    K = cd2d_upwind(47)  # N = 2209: several SpMV blocks and a ragged tail
    A = column_scaled(K, log_uniform(K.n, -3.0, 3.0, seed=11))
    b = randn(K.n, 12)
    h, st, ref = _check_against_oracle(A, b, 1e-9, extra=dict(dia=dia))
    plain = sdr_solve(A.to_scipy(), b, tol=1e-9, max_cycles=ref.cycles + 2, **KW)
    print(f"jacobi: {st['iters']} steps; unpreconditioned after {plain.cycles} cycles: "
          f"relres {plain.relres:.2e}", flush=True)
    assert not plain.converged


def test_jacobi_complex_helmholtz_matches_oracle():
    K = helmholtz2d(40, kappa=10.0)
    A = column_scaled(K, log_uniform(K.n, -2.0, 2.0, seed=13))
    _check_against_oracle(A, crandn(K.n, 14), 1e-9)


def test_jacobi_initial_guess_matches_oracle():
    K = cd2d_upwind(30)
    A = column_scaled(K, log_uniform(K.n, -2.0, 2.0, seed=15))
    x0 = 0.1 * randn(K.n, 16) / log_uniform(K.n, -2.0, 2.0, seed=15)
    _check_against_oracle(A, randn(K.n, 17), 1e-9, x0=x0)


def test_jacobi_sequence_exact_variant_matches_oracle():
    """update_matrix refreshes A D^-1; the recycle space is that of A_i D_i^-1."""
    K = cd2d_upwind(40)
    h = gp._solver(K, precond=1, **KW)
    rec = None
    for i in range(1, 4):
        Ai = column_scaled(K, log_uniform(K.n, -2.0, 2.0, seed=300 + i))
        bi = randn(K.n, 400 + i)
        h.update_matrix(gp._dev(Ai.values))
        x, st = h.solve(gp._dev(bi), tol=1e-9)
        ref = sdr_solve_right_jacobi(Ai.to_scipy(), bi, recycle=rec, new_matrix=True, tol=1e-9, **KW)
        rec = ref.recycle
        gp._assert_trace_and_x(gp._host(x), st, h.trace(), ref, A=Ai, b=bi, tol=1e-9)


def test_jacobi_zero_or_missing_diagonal_is_an_error():
    from paper_2311_14206_amd.sdr import SDRError
    K = cd2d_upwind(12)
    b = gp._dev(randn(K.n, 18))
    rows = np.repeat(np.arange(K.n), np.diff(K.row_ptr))
    zero = K.values.copy()
    zero[np.nonzero(K.col_idx == rows)[0][5]] = 0.0
    h = gp._solver(K.with_values(zero), precond=1, **KW)
    with pytest.raises(SDRError, match="diagonal"):
        h.solve(b, tol=1e-8)
    h = gp._solver(K, precond=1, **KW)
    x, st = h.solve(b, tol=1e-8)
    assert st["converged"]
    with pytest.raises(SDRError, match="diagonal"):
        h.update_matrix(gp._dev(zero))
    # the rejected matrix is not solved with the previous one's A D^-1
    with pytest.raises(SDRError, match="diagonal"):
        h.solve(b, tol=1e-8)
    h.update_matrix(gp._dev(K.values))
    x, st = h.solve(b, tol=1e-8)
    assert st["converged"]


def test_jacobi_with_fp32_basis_reaches_fp64_tolerance():
    """precision=1: A D^-1 narrowed to FP32 for the basis, residuals on the FP64 values."""
    K = cd2d_upwind(47)
    A = column_scaled(K, log_uniform(K.n, -3.0, 3.0, seed=11))
    b = randn(K.n, 12)
    h = gp._solver(A, precond=1, precision=1, **KW)
    x, st = h.solve(gp._dev(b), tol=1e-8)
    xg = gp._host(x)
    assert st["converged"]
    assert np.linalg.norm(b - A.to_scipy() @ xg) <= 1e-8 * np.linalg.norm(b)
    ref = sdr_solve_right_jacobi(A.to_scipy(), b, tol=1e-8, **KW)
    err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    print(f"jacobi + FP32 basis: {st['iters']} steps (oracle {ref.iters}), "
          f"rel. error vs FP64 oracle {err:.2e}", flush=True)
    assert err < 1e-5


def test_spmv_and_adjoint_of_a_preconditioned_handle_use_a():
    """precond applies to the forward solve only: sdr_spmv gives A x and the
    adjoint solve solves A^T lambda = g."""
    K = cd2d_upwind(30)
    A = column_scaled(K, log_uniform(K.n, -1.0, 1.0, seed=19))
    h = gp._solver(A, precond=1, **KW)
    x0 = randn(K.n, 20)
    y = gp._host(h.spmv(gp._dev(x0)))
    ref = A.to_scipy() @ x0
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)
    b = randn(K.n, 21)
    x, st = h.solve(gp._dev(b), tol=1e-9)
    assert st["converged"]
    g = randn(K.n, 22)
    lam, sa = h.solve_adjoint(gp._dev(g), tol=1e-9)
    assert sa["converged"]
    r = g - A.to_scipy().T @ gp._host(lam)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(g)


def test_adjoint_after_a_rejected_preconditioner_update_uses_the_new_matrix():
    """A matrix with a zero diagonal entry is rejected for the preconditioned
    forward solve, but the adjoint solve (which uses A itself) must then work
    on that new matrix, with its recycle space's S A^T U recomputed."""
    from paper_2311_14206_amd.sdr import SDRError
    K = cd2d_upwind(30)
    h = gp._solver(K, precond=1, **KW)
    b = randn(K.n, 24)
    g = randn(K.n, 25)
    x, st = h.solve(gp._dev(b), tol=1e-9)
    lam0, s0 = h.solve_adjoint(gp._dev(g), tol=1e-9)
    assert st["converged"] and s0["converged"]
    rows = np.repeat(np.arange(K.n), np.diff(K.row_ptr))
    zero = K.values.copy()
    zero[np.nonzero(K.col_idx == rows)[0][7]] = 0.0
    with pytest.raises(SDRError, match="diagonal"):
        h.update_matrix(gp._dev(zero))
    Z = K.with_values(zero)
    lam, sa = h.solve_adjoint(gp._dev(g), tol=1e-9)
    assert sa["converged"]
    r = g - Z.to_scipy().T @ gp._host(lam)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(g)
    # the oracle's adjoint sequence: A^T, then the new matrix's transpose
    # with the recycle space carried and S A^T U recomputed
    ref0 = sdr_solve(K.to_scipy().T.tocsr(), g, tol=1e-9, **KW)
    ref = sdr_solve(Z.to_scipy().T.tocsr(), g, recycle=ref0.recycle, new_matrix=True, tol=1e-9, **KW)
    xg = gp._host(lam)
    print(f"adjoint after rejected update: {sa['iters']} steps (oracle {ref.iters}), "
          f"rel. diff {np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x):.1e}", flush=True)
    assert np.linalg.norm(xg - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
