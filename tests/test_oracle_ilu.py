"""Pins of the oracle's ILU(0) right preconditioning (Section 6 preconditions
its Stokes solves by ILU; the variant -- zero fill, right side, greedy
multicolour order -- is the oracle's reading).

References used here, none of them the oracle's own loops: the checkerboard
closed form of a 5-point stencil's greedy colouring, a brute-force colouring
check, the defining property of ILU(0) ((L U)_ij = A_ij on the pattern), an
ILU(0) by column elimination on a dense copy (a different loop order that
must give the same factors), dense solves, and a diagonal matrix, for which
the preconditioner is exact.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ILU0, greedy_colours, ilu0, multicolour_order, sdr_solve, sdr_solve_right_ilu0
from workloads import cd2d_upwind, crandn, helmholtz2d, randn


def _general(n, seed, cplx=False):
    """Nonsymmetric pattern without stencil structure, diagonally shifted."""
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        c = g.choice(n, size=4, replace=False)
        rows.extend([i] * 4)
        cols.extend(c.tolist())
    v = g.standard_normal(len(rows))
    if cplx:
        v = v + 1j * g.standard_normal(len(rows))
    M = sp.csr_matrix((v, (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    return (M + 6.0 * sp.identity(n)).tocsr()


def test_five_point_colouring_is_the_checkerboard():
    n = 9
    A = cd2d_upwind(n).to_scipy()
    c = greedy_colours(A)
    i, j = np.divmod(np.arange(n * n), n)
    assert np.array_equal(c, (i + j) % 2)


def test_colouring_is_proper_and_greedy():
    A = _general(120, 3)
    c = greedy_colours(A)
    S = (abs(A) + abs(A.T)).tocoo()
    for a, b in zip(S.row, S.col):
        if a != b:
            assert c[a] != c[b]
    Sc = S.tocsr()
    for v in range(A.shape[0]):
        lower = {c[u] for u in Sc.indices[Sc.indptr[v]:Sc.indptr[v + 1]] if u < v}
        assert c[v] == min(set(range(len(lower) + 1)) - lower)
    order = multicolour_order(c)
    assert np.all(np.diff(c[order]) >= 0)


def _dense_ilu0_by_columns(Ad, pattern):
    """ILU(0) as Gaussian elimination by columns, dropping every update that
    falls outside the pattern (k outer, i and j inner)."""
    a = Ad.astype(complex if np.iscomplexobj(Ad) else float).copy()
    n = a.shape[0]
    for k in range(n):
        for i in range(k + 1, n):
            if not pattern[i, k]:
                continue
            a[i, k] /= a[k, k]
            for j in range(k + 1, n):
                if pattern[i, j] and pattern[k, j]:
                    a[i, j] -= a[i, k] * a[k, j]
    L = np.tril(a, -1) + np.eye(n)
    U = np.triu(a)
    return L * (pattern | np.eye(n, dtype=bool)), U * pattern


@pytest.mark.parametrize("kind", ["cd", "general", "complex"])
def test_ilu0_defining_property_and_column_elimination(kind):
    if kind == "cd":
        A = cd2d_upwind(7).to_scipy()
    elif kind == "general":
        A = _general(60, 5)
    else:
        A = _general(50, 6, cplx=True)
    M = ILU0(A)
    Ap = A[M.order][:, M.order].tocsr()
    L, U = M.L.toarray(), M.U.toarray()
    pattern = Ap.toarray() != 0
    np.fill_diagonal(pattern, True)
    n = A.shape[0]
    # L unit lower, U upper, both on the pattern
    assert np.allclose(np.diag(L), 1.0)
    assert np.all(L[np.triu_indices(n, 1)] == 0) and np.all(U[np.tril_indices(n, -1)] == 0)
    off = ~pattern
    assert np.all(L[off] == 0) and np.all(U[off] == 0)
    # (L U)_ij = A_ij on the pattern
    LU = L @ U
    scale = np.abs(Ap.toarray()).max()
    assert np.max(np.abs((LU - Ap.toarray())[pattern])) <= 1e-13 * scale
    # same factors as elimination by columns
    Lc, Uc = _dense_ilu0_by_columns(Ap.toarray(), pattern)
    assert np.max(np.abs(L - Lc)) <= 1e-12 and np.max(np.abs(U - Uc)) <= 1e-12 * scale


def test_apply_and_multiply_are_inverse_and_match_dense_factors():
    A = _general(80, 9)
    M = ILU0(A)
    v = randn(80, 1)
    z = M.solve(v)
    assert np.linalg.norm(M.mult(z) - v) <= 1e-13 * np.linalg.norm(v)
    P = np.eye(80)[M.order]
    Md = P.T @ (M.L.toarray() @ M.U.toarray()) @ P
    assert np.linalg.norm(Md @ z - v) <= 1e-13 * np.linalg.norm(v)


def test_zero_pivot_raises():
    A = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]]))
    with pytest.raises(ValueError, match="pivot"):
        ILU0(A)
    with pytest.raises(ValueError, match="pivot"):
        ilu0(A)


def test_diagonal_matrix_is_solved_in_one_step():
    """For a diagonal A the ILU(0) is A itself: A M^-1 = I, one Arnoldi step."""
    d = np.linspace(1.0, 5.0, 200)
    A = sp.diags(d).tocsr()
    b = randn(200, 2)
    r = sdr_solve_right_ilu0(A, b, m=10, k=2, t=2, s=32, tol=1e-12)
    assert r.converged and r.iters == 1
    assert np.linalg.norm(r.x - b / d) <= 1e-14 * np.linalg.norm(b / d)


@pytest.mark.parametrize("kind", ["cd", "helmholtz"])
def test_preconditioned_solution_matches_dense_solve(kind):
    if kind == "cd":
        A = cd2d_upwind(24).to_scipy()
        b = randn(A.shape[0], 4)
    else:
        A = helmholtz2d(20, kappa=6.0).to_scipy()
        b = crandn(A.shape[0], 4)
    x0 = 0.1 * (randn(A.shape[0], 5) if kind == "cd" else crandn(A.shape[0], 5))
    r = sdr_solve_right_ilu0(A, b, x0=x0, m=20, k=5, t=2, s=64, tol=1e-10)
    assert r.converged
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(b - A @ r.x) <= 1e-10 * np.linalg.norm(b)
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(r.x - xd) <= 10 * cond * 1e-10 * np.linalg.norm(xd)
    # preconditioning pays: fewer steps than the plain method
    p = sdr_solve(A, b, x0=x0, m=20, k=5, t=2, s=64, tol=1e-10)
    assert r.iters < p.iters
