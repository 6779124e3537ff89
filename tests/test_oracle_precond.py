"""Pins of the oracle's right Jacobi preconditioned solve.

Right preconditioning (Section 6 runs its Stokes systems preconditioned) in
its diagonal form: A x = b is solved as (A D^-1) u = b, x = D^-1 u, with
D = diag(A).  The pins below do not restate that formula; they check it
against what it implies:

* for A = K diag(c) with powers of two c_j, every product and quotient of
  A D^-1 is exact, so A D^-1 equals K diag(1/kappa) (kappa = diag(K)) bit for
  bit; the preconditioned solve on A must then take the unpreconditioned
  solve on K diag(1/kappa) step for step, with x = y / (kappa c).  Left
  instead of right scaling, D instead of D^-1, or a missing x = D^-1 u each
  break this;
* a diagonal A gives A D^-1 = I: one step, x = b / d;
* the true residual of A x = b meets the tolerance;
* an exact initial guess is returned as it is, without a cycle.
"""

import numpy as np
import pytest

from oracle import sdr_solve, sdr_solve_right_jacobi
from workloads import CSR, cd2d_upwind, column_scaled, crandn, helmholtz2d, log_uniform, randn

P = dict(m=30, k=6, t=2, s=80, max_cycles=40)  # the unmutated solves take 2 or 3 cycles


def _diag(A):
    return A.to_scipy().diagonal()


@pytest.mark.parametrize("cplx", [False, True])
def test_power_of_two_columns_reduce_to_the_unscaled_solve(cplx):
    K = helmholtz2d(18, kappa=8.0) if cplx else cd2d_upwind(20)
    c = log_uniform(K.n, -3.0, 3.0, seed=7, pow2=True)
    A = column_scaled(K, c)
    kappa = _diag(K)
    B = column_scaled(K, 1.0 / kappa)
    b = crandn(K.n, 3) if cplx else randn(K.n, 3)
    pre = sdr_solve_right_jacobi(A.to_scipy(), b, tol=1e-8, **P)
    ref = sdr_solve(B.to_scipy(), b, tol=1e-8, **P)
    assert pre.converged and ref.converged
    assert [c_.j_stop for c_ in pre.trace] == [c_.j_stop for c_ in ref.trace]
    assert [c_.k_eff for c_ in pre.trace] == [c_.k_eff for c_ in ref.trace]
    for cp, cr in zip(pre.trace, ref.trace):
        assert cp.res == cr.res
    assert (pre.iters, pre.matvecs, pre.inner_products) == (ref.iters, ref.matvecs, ref.inner_products)
    np.testing.assert_allclose(pre.x, ref.x / (kappa * c), rtol=1e-14, atol=0)
    r = b - A.to_scipy() @ pre.x
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)


def test_diagonal_matrix_is_one_step():
    import scipy.sparse as sp
    d = log_uniform(500, -4.0, 4.0, seed=3) * np.where(randn(500, 4) > 0, 1.0, -1.0)
    A = CSR.from_scipy(sp.diags(d).tocsr())
    b = randn(500, 5)
    out = sdr_solve_right_jacobi(A.to_scipy(), b, tol=1e-10, m=10, k=2, t=2, s=32)
    assert out.converged and out.cycles == 1 and out.iters == 1
    np.testing.assert_allclose(out.x, b / d, rtol=1e-13, atol=0)
    # unpreconditioned, the same system needs many steps
    plain = sdr_solve(A.to_scipy(), b, tol=1e-10, m=10, k=2, t=2, s=32, max_cycles=3)
    assert plain.iters > 10


def test_badly_scaled_columns_converge_as_the_balanced_system():
    K = cd2d_upwind(20)
    c = log_uniform(K.n, -3.0, 3.0, seed=11)
    A = column_scaled(K, c)
    b = randn(K.n, 12)
    pre = sdr_solve_right_jacobi(A.to_scipy(), b, tol=1e-8, **P)
    bal = sdr_solve(column_scaled(K, 1.0 / _diag(K)).to_scipy(), b, tol=1e-8, **P)
    plain = sdr_solve(A.to_scipy(), b, tol=1e-8, **{**P, "max_cycles": 5})
    assert pre.converged
    assert abs(pre.iters - bal.iters) <= P["m"]
    assert not plain.converged or plain.iters > 2 * pre.iters
    r = b - A.to_scipy() @ pre.x
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)


def test_exact_initial_guess_and_zero_diagonal():
    K = cd2d_upwind(12)
    A = column_scaled(K, log_uniform(K.n, -2.0, 2.0, seed=5))
    xs = randn(K.n, 6)
    b = A.to_scipy() @ xs
    out = sdr_solve_right_jacobi(A.to_scipy(), b, x0=xs, tol=1e-8, **P)
    assert out.converged and out.cycles == 0
    np.testing.assert_allclose(out.x, xs, rtol=1e-15, atol=0)
    As = A.to_scipy().tolil()
    As[4, 4] = 0.0
    with pytest.raises(ValueError):
        sdr_solve_right_jacobi(As.tocsr(), b, tol=1e-8, **P)
