"""GPU parity of the subsampled randomised DCT sketch (option sketch=1,
Section 6) against the oracle's SRDCT (scipy's orthonormal DCT-II on the same
signs and rows): the operator itself to 1e-12, at small and full size, and
complete solves (decision traces and x) with it."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import SRDCT, sdr_solve
from workloads import CSR, cd2d_upwind, crandn, helmholtz2d, randn, shifted_diagonal, workload

import test_gpu_parity as gp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _identity_handle(N, s, seed, cplx):
    dt = np.complex128 if cplx else np.float64
    A = CSR.from_scipy(sp.identity(N, dtype=dt, format="csr"))
    return gp._solver(A, m=4, k=1, t=2, s=s, seed=seed, sketch=1)


@pytest.mark.parametrize("N,s,cplx", [(5000, 120, False), (777, 48, False), (4099, 96, True),
                                      (1536, 1536, False)])
def test_dct_sketch_operator_matches_oracle(N, s, cplx):
    """S X against scipy's DCT of E X, rows P, scale sqrt(N/s); with s = N
    every row is kept and S is orthogonal."""
    h = _identity_handle(N, s, 777, cplx)
    g = np.random.default_rng(N)
    X = g.standard_normal((N, 3))
    if cplx:
        X = X + 1j * g.standard_normal((N, 3))
    Y = gp._host(h.sketch(gp._dev(X)))
    ref = SRDCT(N, s, 777) @ X
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    print(f"[gpu] DCT sketch N={N} s={s} complex={cplx}: rel. diff {err:.1e}", flush=True)
    assert err <= 1e-12
    if s == N:
        assert abs(np.linalg.norm(Y[:, 0]) - np.linalg.norm(X[:, 0])) <= 1e-12 * np.linalg.norm(X[:, 0])


def test_dct_sketch_full_size():
    """N = 2^20, s = 240: every row of S x to 1e-12 of the largest."""
    N, s = 1 << 20, 240
    h = _identity_handle(N, s, 42, False)
    x = randn(N, 5)
    y = gp._host(h.sketch(gp._dev(x)))
    ref = SRDCT(N, s, 42) @ x
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    print(f"[gpu] DCT sketch N=2^20: max rel. diff {err:.1e}", flush=True)
    assert err <= 1e-12


def _compare(A, b, kw, tol, **extra):
    h = gp._solver(A, sketch=1, **kw, **extra)
    x, st = h.solve(gp._dev(b), tol=tol)
    ref = sdr_solve(A.to_scipy(), b, tol=tol, sketch="srdct", **kw)
    gp._assert_trace_and_x(gp._host(x), st, h.trace(), ref, A=A, b=b, tol=tol)
    return h, st, ref


@pytest.mark.parametrize("dia", [1, 0])
def test_dct_solve_cd2d_64_matches_oracle(dia):
    A, b, p = workload("cd2d_64")
    _compare(A, b, dict(m=p["m"], k=p["k"], t=p["t"], s=p["s"]), p["tol"], dia=dia)


def test_dct_solve_complex_helmholtz_matches_oracle():
    A = helmholtz2d(32, kappa=8.0)
    _compare(A, crandn(A.n, 3), dict(m=40, k=8, t=3, s=96), 1e-9)


def test_dct_sequence_exact_variant_matches_oracle():
    A0 = cd2d_upwind(40)
    kw = dict(m=30, k=6, t=2, s=80)
    h = gp._solver(A0, sketch=1, **kw)
    rec = None
    for i in range(1, 4):
        d = 1e-2 * np.random.default_rng(100 + i).uniform(0, 1, A0.n)
        Ai = shifted_diagonal(A0, d)
        bi = randn(A0.n, 200 + i)
        h.update_matrix(gp._dev(Ai.values))
        x, st = h.solve(gp._dev(bi), tol=1e-9)
        ref = sdr_solve(Ai.to_scipy(), bi, recycle=rec, new_matrix=True, tol=1e-9, sketch="srdct", **kw)
        rec = ref.recycle
        gp._assert_trace_and_x(gp._host(x), st, h.trace(), ref, A=Ai, b=bi, tol=1e-9)


def test_dct_with_fp32_basis_reaches_fp64_tolerance():
    A, b, p = workload("cd2d_64")
    h = gp._solver(A, m=p["m"], k=p["k"], t=p["t"], s=p["s"], sketch=1, precision=1)
    x, st = h.solve(gp._dev(b), tol=1e-8)
    xg = gp._host(x)
    assert st["converged"]
    assert np.linalg.norm(b - A.to_scipy() @ xg) <= 1e-8 * np.linalg.norm(b)
    ref = sdr_solve(A.to_scipy(), b, m=p["m"], k=p["k"], t=p["t"], s=p["s"], tol=1e-8, sketch="srdct")
    err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    print(f"DCT sketch + FP32 basis: {st['iters']} steps (oracle {ref.iters}), "
          f"rel. error vs FP64 oracle {err:.2e}", flush=True)
    assert err < 1e-5
