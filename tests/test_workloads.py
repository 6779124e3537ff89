"""Input generators: stencils against dense assembly, nnz closed forms."""

import numpy as np
import scipy.sparse as sp

from workloads import (cd2d_upwind, cd3d_upwind, helmholtz2d, cd2d_central,
                       theta_weighted, shifted_diagonal, randn, crandn, workload)


def _dense_1d(n, lo, di, up):
    return np.diag(np.full(n, di)) + np.diag(np.full(n - 1, lo), -1) + np.diag(np.full(n - 1, up), 1)


def test_nnz_closed_forms():
    for n in (3, 7, 16):
        assert cd2d_upwind(n).nnz == 5 * n * n - 4 * n
        assert cd3d_upwind(n).nnz == 7 * n ** 3 - 6 * n * n
        assert helmholtz2d(n).nnz == 5 * n * n - 4 * n


def test_cd2d_upwind_matches_kron_assembly():
    n = 9
    h = 1.0 / (n + 1)
    bx, by = 50.0, 50.0
    # -Laplace via 1D second differences, upwind first differences, times h^2
    T = _dense_1d(n, -1.0, 2.0, -1.0)
    Dup = _dense_1d(n, -1.0, 1.0, 0.0)  # backward difference (u_i - u_{i-1})
    I = np.eye(n)
    ref = np.kron(I, T) + np.kron(T, I) + h * bx * np.kron(I, Dup) + h * by * np.kron(Dup, I)
    A = cd2d_upwind(n).to_scipy().toarray()
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-14)


def test_cd3d_upwind_matches_kron_assembly():
    n = 5
    h = 1.0 / (n + 1)
    b = 50.0
    T = _dense_1d(n, -1.0, 2.0, -1.0)
    D = _dense_1d(n, -1.0, 1.0, 0.0)
    I = np.eye(n)
    K = lambda a, c, d: np.kron(a, np.kron(c, d))
    ref = (K(I, I, T) + K(I, T, I) + K(T, I, I)
           + h * b * (K(I, I, D) + K(I, D, I) + K(D, I, I)))
    A = cd3d_upwind(n).to_scipy().toarray()
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-14)


def test_helmholtz_and_central_match_kron():
    n = 6
    h = 1.0 / (n + 1)
    T = _dense_1d(n, -1.0, 2.0, -1.0)
    I = np.eye(n)
    kap = 20.0
    ref = np.kron(I, T) + np.kron(T, I) - (kap * h) ** 2 * (1 + 0.5j) * np.eye(n * n)
    np.testing.assert_allclose(helmholtz2d(n, kap).to_scipy().toarray(), ref, atol=1e-14)
    L = (n + 1) ** 2 * _dense_1d(n, 1.0, -2.0, 1.0)
    D = (n + 1) / 2.0 * _dense_1d(n, -1.0, 0.0, 1.0)
    alpha = 5.0
    ref = np.kron(L, I) + np.kron(I, L) + alpha * (np.kron(D, I) + np.kron(I, D))
    np.testing.assert_allclose(cd2d_central(n, alpha).to_scipy().toarray(), ref, rtol=1e-14,
                               atol=1e-9)


def test_csr_invariants_and_helpers():
    A = cd2d_upwind(8)
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32
    for i in range(A.n):
        c = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    th = 1 + 0.1 * randn(A.nnz, 7)
    At = theta_weighted(A, th)
    np.testing.assert_array_equal(At.values, th * A.values)
    d = np.arange(A.n, dtype=float)
    As = shifted_diagonal(A, d).to_scipy().toarray()
    np.testing.assert_allclose(As - A.to_scipy().toarray(), np.diag(d), atol=1e-15)


def test_seeded_vectors():
    a = randn(10, 1)
    np.testing.assert_array_equal(a, np.random.default_rng(1).standard_normal(10))
    c = crandn(10000, 3)
    assert abs(np.mean(np.abs(c) ** 2) - 1.0) < 0.05
    A, b, p = workload("cd2d_64")
    assert A.n == 4096 and A.nnz == 20224 and b.shape == (4096,)
    assert p["s"] == 2 * (p["m"] + p["k"])
