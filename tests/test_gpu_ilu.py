"""GPU parity of right ILU(0) preconditioning (option "precond" 2) against the oracle.

Section 6 preconditions by ILU; the library and the oracle both take ILU(0)
on A's pattern in a greedy multicolour elimination order, applied on the
right ((A M^-1) u = b, x = M^-1 u), each written from that definition.  The
apply M^-1 v is checked alone to rounding, then complete solves by their
decision traces and x: convection-diffusion (two colours, diagonal and CSR
storage, a ragged tail), complex Helmholtz, a general pattern with many
colours and long rows, a nonzero initial guess, the FP32 basis, a sequence
that refactors on update_matrix, and the zero-pivot error path.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ILU0, sdr_solve, sdr_solve_right_ilu0
from workloads import CSR, cd2d_upwind, crandn, helmholtz2d, randn

import test_gpu_parity as gp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KW = dict(m=30, k=6, t=2, s=80)


def _general(n, seed):
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = 120 if 50 <= i < 53 else 5
        c = g.choice(n, size=k, replace=False)
        rows.extend([i] * k)
        cols.extend(c.tolist())
    M = sp.csr_matrix((g.standard_normal(len(rows)), (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    return CSR.from_scipy((M + 8.0 * sp.identity(n)).tocsr())


def _check(A, b, tol, x0=None, extra=None, kw=KW, strict=True):
    h = gp._solver(A, precond=2, **kw, **(extra or {}))
    x, st = h.solve(gp._dev(b), x=None if x0 is None else gp._dev(x0), tol=tol)
    ref = sdr_solve_right_ilu0(A.to_scipy(), b, x0=x0, tol=tol, **kw)
    xg = gp._host(x)
    print(f"ilu(0): {st['iters']} steps (oracle {ref.iters}), {len(ILU0(A.to_scipy()).order) and ''}"
          f"colours {int(ILU0(A.to_scipy()).colours.max()) + 1}", flush=True)
    gp._assert_trace_and_x(xg, st, h.trace(), ref, A=A, b=b, tol=tol, strict=strict)
    r = b - A.to_scipy() @ xg
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b)
    return h, st, ref


@pytest.mark.parametrize("kind", ["cd", "helmholtz", "general"])
def test_ilu_apply_matches_oracle(kind):
    if kind == "cd":
        A = cd2d_upwind(45)
        v = randn(A.n, 21)
    elif kind == "helmholtz":
        A = helmholtz2d(37, kappa=9.0)
        v = crandn(A.n, 22)
    else:
        A = _general(700, 23)
        v = randn(A.n, 24)
    h = gp._solver(A, precond=2, **KW)
    z = gp._host(h.precond_apply(gp._dev(v)))
    M = ILU0(A.to_scipy())
    zo = M.solve(v)
    d = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    print(f"[gpu] ILU(0) apply {kind} n={A.n} colours={int(M.colours.max()) + 1}: rel. diff {d:.1e}", flush=True)
    assert d <= 1e-13


@pytest.mark.parametrize("dia", [1, 0])
def test_ilu_cd2d_matches_oracle(dia):
    A = cd2d_upwind(47)
    b = randn(A.n, 25)
    h, st, ref = _check(A, b, 1e-9, extra=dict(dia=dia))
    plain = sdr_solve(A.to_scipy(), b, tol=1e-9, **KW)
    print(f"ilu(0) {st['iters']} steps, unpreconditioned {plain.iters}", flush=True)
    assert st["iters"] < plain.iters


def test_ilu_complex_helmholtz_matches_oracle():
    A = helmholtz2d(40, kappa=10.0)
    _check(A, crandn(A.n, 26), 1e-9)


def test_ilu_general_pattern_matches_oracle():
    A = _general(1500, 27)
    _check(A, randn(A.n, 28), 1e-9)


def test_ilu_initial_guess_matches_oracle():
    A = cd2d_upwind(30)
    _check(A, randn(A.n, 29), 1e-9, x0=0.1 * randn(A.n, 30))


def test_ilu_fp32_basis_reaches_the_tolerance():
    A = cd2d_upwind(47)
    b = randn(A.n, 31)
    h = gp._solver(A, precond=2, precision=1, **KW)
    x, st = h.solve(gp._dev(b), tol=1e-8)
    ref = sdr_solve_right_ilu0(A.to_scipy(), b, tol=1e-8, **KW)
    xg = gp._host(x)
    assert st["converged"]
    assert np.linalg.norm(b - A.to_scipy() @ xg) <= 1e-8 * np.linalg.norm(b)
    print(f"ilu(0) fp32 basis: {st['iters']} steps (fp64 oracle {ref.iters}), x rel. error vs oracle "
          f"{np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x):.1e}", flush=True)


def test_ilu_sequence_refactors_on_update():
    """update_matrix refactors M; the recycle space belongs to A_i M_i^-1."""
    K = cd2d_upwind(40)
    h = gp._solver(K, precond=2, **KW)
    rec = None
    for i in range(1, 4):
        d = 1e-1 * np.random.default_rng(500 + i).uniform(0, 1, K.n)
        from workloads import shifted_diagonal
        Ai = shifted_diagonal(K, d)
        bi = randn(K.n, 600 + i)
        h.update_matrix(gp._dev(Ai.values))
        x, st = h.solve(gp._dev(bi), tol=1e-9)
        ref = sdr_solve_right_ilu0(Ai.to_scipy(), bi, recycle=rec, new_matrix=True, tol=1e-9, **KW)
        rec = ref.recycle
        gp._assert_trace_and_x(gp._host(x), st, h.trace(), ref, A=Ai, b=bi, tol=1e-9)


def test_ilu_zero_pivot_is_an_error_until_a_valid_matrix():
    from paper_2311_14206_amd.sdr import SDRError
    K = cd2d_upwind(12)
    b = gp._dev(randn(K.n, 32))
    rows = np.repeat(np.arange(K.n), np.diff(K.row_ptr))
    bad = K.values.copy()
    bad[np.nonzero(K.col_idx == rows)[0][0]] = 0.0  # row 0 (colour 0): a zero pivot
    h = gp._solver(K, precond=2, **KW)
    x, st = h.solve(b, tol=1e-9)
    assert st["converged"]
    with pytest.raises(SDRError):
        h.update_matrix(gp._dev(bad))
    with pytest.raises(SDRError):
        h.solve(b, tol=1e-9)
    h.update_matrix(gp._dev(K.values))
    x, st = h.solve(b, tol=1e-9)
    assert st["converged"]
