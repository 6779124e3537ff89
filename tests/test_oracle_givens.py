"""Pins of the oracle's Givens-rotation residual control (Sections 4.5 and 5).

* The sketched residual norms of the sketched least squares satisfy
  ||S r_j|| = |s_j| ||S r_{j-1}|| with s_j the j-th Givens sine of the QR
  factorisation of the augmented Hessenberg matrix G_j (the Givens-sine
  theorem of Section 4.5, extended to [U V] in Section 5).  The oracle builds
  G_j and rotates it; the reference is the minimum of an independent lstsq.
* With S = I the sketched sines are the true ones, so the estimate with
  eps = 0 is the true residual of every iterate (the textbook GMRES residual
  recursion) and the first true-residual check is the first step below the
  tolerance.
* With a real sketch and eps the exact distortion of S on the cycle's space,
  the corollary's bound ||r_j|| <= sqrt((s_j^2 + 2 eps (1 + c_j)) /
  (1 - eps^2)) ||r_{j-1}|| (unsketched sines s_j, c_j) holds for the oracle's
  iterates (Fig. 3 plots this estimate).
* The eps refit after a failed check makes the estimate from the previous
  anchor reach the observed true residual, and eps never decreases.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import sdr_solve
from oracle.gmres_sdr import givens_sine, givens_factor, sketched_least_squares
from oracle.sketch import sketch_operator
from workloads import cd2d_upwind, helmholtz2d, randn, crandn


def _cycles(A, b, S, m, k, t, s, max_cycles=3, tol=1e-14):
    keep = []
    r = sdr_solve(A, b, m=m, k=k, t=t, s=s, S=S, tol=tol, max_cycles=max_cycles, keep_cycles=keep)
    return r, keep


@pytest.mark.parametrize("cplx", [False, True])
def test_sketched_residual_is_givens_sine_times_previous(cplx):
    """||S r_j|| = |s_j| ||S r_{j-1}|| in every step of cycles with and
    without a recycled block (Section 4.5 theorem; Section 5 for [U V])."""
    if cplx:
        A = helmholtz2d(14, kappa=5.0).to_scipy()
        b = crandn(A.shape[0], 4)
    else:
        A = cd2d_upwind(14).to_scipy()
        b = randn(A.shape[0], 4)
    N = A.shape[0]
    S = sketch_operator(N, 96, 8, 5)
    r, keep = _cycles(A, b, S, m=20, k=5, t=2, s=96)
    assert len(keep) >= 2 and keep[1]["U_in"].shape[1] > 0
    for kc, rec in zip(keep, r.trace):
        SAU, Sr = kc["SAU_in"], kc["Sr"]
        prev = sketched_least_squares(SAU, Sr)[1] if SAU.shape[1] else np.linalg.norm(Sr)
        for j in range(1, kc["j"] + 1):
            sj = givens_sine(SAU, kc["SV"], kc["H"], j)
            assert 0.0 <= sj <= 1.0
            assert abs(sj * prev - rec.sres_hist[j - 1]) <= 1e-10 * prev, (j, sj * prev, rec.sres_hist[j - 1])
            prev = rec.sres_hist[j - 1]


def test_identity_sketch_estimate_is_the_true_residual():
    """S = I, full orthogonalisation: every estimate equals the true residual
    of its iterate, the first check comes at the first step whose GMRES
    residual (dense lstsq over the Krylov matrix) is below tol, and it
    converges; eps is never raised."""
    A = cd2d_upwind(10).to_scipy()
    N = A.shape[0]
    b = randn(N, 6)
    m, tol = 12, 1e-8
    r = sdr_solve(A, b, m=m, k=4, t=m, s=N, S=sp.identity(N, format="csr"), tol=tol,
                  resid_control="givens")
    assert r.converged and r.eps <= 1e-12
    assert len(r.trace) >= 3  # later cycles start from a recycled block
    # cycle 1 from x0 = 0: dense GMRES residuals by step
    Ad = A.toarray()
    # orthonormal Krylov basis by Arnoldi with two Gram-Schmidt passes
    Q = np.zeros((N, m))
    Q[:, 0] = b / np.linalg.norm(b)
    for j in range(1, m):
        w = Ad @ Q[:, j - 1]
        for _ in range(2):
            w -= Q[:, :j] @ (Q[:, :j].T @ w)
        Q[:, j] = w / np.linalg.norm(w)
    gm = []
    for j in range(1, m + 1):
        y, *_ = np.linalg.lstsq(Ad @ Q[:, :j], b, rcond=None)
        gm.append(np.linalg.norm(b - Ad @ Q[:, :j] @ y))
    tol_abs = tol * np.linalg.norm(b)
    for c in r.trace:
        for ch in c.checks:
            assert abs(ch.est - ch.res) <= 1e-9 * ch.res, (ch.est, ch.res)
    below = [j for j in range(1, m + 1) if gm[j - 1] < tol_abs]
    first = r.trace[0]
    if below:
        assert len(first.checks) == 1 and first.checks[0].j == below[0] and first.converged
    else:
        assert [ch.j for ch in first.checks] == [m]
    # (a check that is not the cycle's last is a converged one)
    assert all(len(c.checks) == 1 for c in r.trace)
    # a new right-hand side with the recycle space carried: the first cycle
    # starts from the sketched minimiser over span(U), whose true residual the
    # estimate must also reproduce
    b2 = randn(N, 16)
    r2 = sdr_solve(A, b2, m=m, k=4, t=m, s=N, S=sp.identity(N, format="csr"), tol=tol,
                   resid_control="givens", recycle=r.recycle)
    assert r2.converged and r2.eps <= 1e-12
    for c in r2.trace:
        for ch in c.checks:
            assert abs(ch.est - ch.res) <= 1e-9 * ch.res, (ch.est, ch.res)


def test_corollary_bound_with_exact_epsilon():
    """||r_j|| <= sqrt((s_j^2 + 2 eps (1+c_j)) / (1 - eps^2)) ||r_{j-1}|| with
    eps the exact distortion of S on span([r0, A W]) and the unsketched sines
    of the angle between r_{j-1} and A [U, V_j] (Section 4.5 corollary)."""
    A = cd2d_upwind(12).to_scipy()
    N = A.shape[0]
    b = randn(N, 7)
    S = sketch_operator(N, 160, 8, 42)
    r, keep = _cycles(A, b, S, m=14, k=4, t=2, s=160, max_cycles=2)
    for kc in keep:
        r0, U, V, j = kc["r0"], kc["U_in"], kc["V"], kc["j"]
        W = np.concatenate([U, V[:, :j]], axis=1)
        Q = sla.orth(np.concatenate([r0[:, None], A @ W], axis=1))
        sv = np.linalg.svd(S @ Q, compute_uv=False)
        eps = max(sv[0] ** 2 - 1, 1 - sv[-1] ** 2)
        assert eps < 1
        SAW = np.concatenate([kc["SAU_in"], kc["SAV"]], axis=1)
        kh = U.shape[1]
        # residual of the sketched minimiser over span(U) (j = 0), then by step
        def resid(jj):
            if kh + jj == 0:
                return r0
            y, _ = sketched_least_squares(SAW[:, : kh + jj], kc["Sr"])
            return r0 - A @ (W[:, : kh + jj] @ y)
        prev = resid(0)
        for jj in range(1, j + 1):
            cur = resid(jj)
            Qj = sla.orth(A @ W[:, : kh + jj])
            p = prev - Qj @ (Qj.T @ prev)
            sn = np.linalg.norm(p) / np.linalg.norm(prev)
            cs = np.sqrt(max(0.0, 1 - sn * sn))
            bound = np.sqrt((sn * sn + 2 * eps * (1 + cs)) / (1 - eps * eps)) * np.linalg.norm(prev)
            assert np.linalg.norm(cur) <= bound * (1 + 1e-10), (jj, np.linalg.norm(cur), bound)
            prev = cur


def test_eps_refit_reaches_the_observed_residual():
    """After each check that exceeds its estimate, the refitted eps is the
    smallest for which the estimate rebuilt from the previous anchor reaches
    that true residual (to the bisection's resolution); eps never decreases
    and the checks record it."""
    A = cd2d_upwind(24).to_scipy()
    N = A.shape[0]
    b = randn(N, 8)
    r = sdr_solve(A, b, m=40, k=8, t=2, s=104, tol=1e-9, resid_control="givens")
    assert r.converged and r.refits
    for res, e0, e1, est_hi, est_lo in r.refits:
        assert e1 > e0
        assert est_hi >= res > est_lo
        assert e1 - np.nextafter(e1, 0) >= 0  # (a representable bracket)
    eps_seq = [ch.eps for c in r.trace for ch in c.checks] + [r.eps]
    assert all(e2 >= e1 for e1, e2 in zip(eps_seq[:-1], eps_seq[1:]))
    assert r.eps == r.refits[-1][2]


def test_givens_control_solution_matches_dense_lu():
    for A, b in ((cd2d_upwind(16).to_scipy(), randn(256, 9)),
                 (helmholtz2d(12, kappa=4.0).to_scipy(), crandn(144, 9))):
        tol = 1e-10
        r = sdr_solve(A, b, m=20, k=5, t=2, s=64, tol=tol, resid_control="givens")
        assert r.converged
        Ad = A.toarray()
        assert np.linalg.norm(b - Ad @ r.x) <= tol * np.linalg.norm(b)
        x = np.linalg.solve(Ad, b)
        assert np.linalg.norm(r.x - x) <= np.linalg.cond(Ad) * tol * np.linalg.norm(x)


def test_givens_factor_special_values():
    """eps = 0: the factor is the sine itself; a sine of 1 (no progress) with
    eps > 0 grows the estimate."""
    for sn in (0.0, 0.3, 0.99, 1.0):
        assert givens_factor(sn, 0.0) == pytest.approx(sn, abs=1e-15)
    assert givens_factor(1.0, 0.1) > 1.0
