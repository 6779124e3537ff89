"""Pins of the GMRES-SDR oracle against facts the paper and the mathematics fix.

Each test names the passage it relies on.  None re-types the oracle's own
formulas: the references are dense textbook computations (lstsq over an
explicit Krylov matrix, dense generalised eigenproblems, LU solves), exact
invariants, or closed-form special cases.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import Recycle, harmonic_ritz_update, sdr_solve
from oracle.sketch import sketch_operator
from workloads import cd2d_upwind, helmholtz2d, randn, crandn, shifted_diagonal


def _orth(X):
    """Orthonormal basis of range(X) (rank-revealing, via the SVD)."""
    return sla.orth(X)


def _max_sin_angle(X, Y):
    """Largest principal-angle sine between range(X) and range(Y), computed as
    the norm of the projection residual (accurate for tiny angles)."""
    Qx, Qy = _orth(X), _orth(Y)
    a = np.linalg.norm(Qy - Qx @ (Qx.conj().T @ Qy), 2)
    b = np.linalg.norm(Qx - Qy @ (Qy.conj().T @ Qx), 2)
    return float(max(a, b))


def _random_nonsym(N, seed, shift=3.0):
    g = np.random.default_rng(seed)
    return shift * np.eye(N) + g.standard_normal((N, N)) / np.sqrt(N)


def _small_cd(n=12):
    return cd2d_upwind(n).to_scipy()


# ---------------------------------------------------------------- Arnoldi --
@pytest.mark.parametrize("cplx", [False, True])
def test_truncated_arnoldi_relation_and_band(cplx):
    """A V_j = V_{j+1} H_j (eq. (2.1) for the truncated process) with H banded
    to t+1 diagonals; the t-window is orthonormal, older vectors are not
    (Algorithm 1, truncated Arnoldi; Section 3.2).  The complex case pins the
    conjugation H(i,j) = V(:,i)^* w."""
    t = 2
    if cplx:  # non-normal complex operator (upwind convection, complex shift)
        A = _small_cd(14).astype(np.complex128)
        A = A + sp.diags(0.5j * np.random.default_rng(4).uniform(0, 1, A.shape[0]))
        b = crandn(A.shape[0], 1)
    else:
        A = _small_cd(14)
        b = randn(A.shape[0], 1)
    keep = []
    sdr_solve(A, b, m=30, k=5, t=t, s=80, tol=1e-14, max_cycles=1, keep_cycles=keep)
    V, H = keep[0]["V"], keep[0]["H"]
    j = H.shape[1]
    lhs = A @ V[:, :j]
    rhs = V @ H
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * sla.norm(A.toarray(), 2) * np.sqrt(j)
    # band: H(i, j) = 0 unless j-t+1 <= i <= j+1 (1-based)
    for jj in range(j):
        for ii in range(H.shape[0]):
            if ii < jj - t + 1 or ii > jj + 1:
                assert H[ii, jj] == 0.0
    G = V.conj().T @ V
    for a in range(V.shape[1]):
        assert abs(G[a, a] - 1) < 1e-14
        for d in range(1, t + 1):
            if a + d < V.shape[1]:
                assert abs(G[a, a + d]) < 1e-13
    # truncation really truncates: far-apart vectors are not orthogonal
    assert np.max(np.abs(np.triu(G, t + 1))) > 1e-6


def test_inner_product_count_is_t_plus_one_per_step():
    """Each truncated Arnoldi step costs min(j, t) window products and one
    norm: about t+1 inner products per matrix-vector product, the ratio seen in
    the tables of Section 6 for t = 2."""
    A = _small_cd(16)
    b = randn(A.shape[0], 2)
    for t in (1, 2, 3):
        r = sdr_solve(A, b, m=25, k=5, t=t, s=64, tol=1e-10, max_cycles=1)
        j = r.iters
        arnoldi_ip = sum(min(i, t) + 1 for i in range(1, j + 1))
        # + ||b - A x0|| + beta of the cycle + one norm per true-residual check
        assert r.inner_products == arnoldi_ip + 2 + r.res_checks


def test_sketch_of_Av_from_arnoldi_relation():
    """SAV(:, j) = SV(:, 1:j+1) H(1:j+1, j) equals the explicit sketch S (A v_j)
    (Section 3: each basis vector is sketched once, and S A v_j follows from
    the Arnoldi relation)."""
    A = _small_cd(14)
    N = A.shape[0]
    b = randn(N, 2)
    S = sketch_operator(N, 80, 8, 42)
    keep = []
    sdr_solve(A, b, m=25, k=5, t=2, s=80, tol=1e-14, max_cycles=1, S=S, keep_cycles=keep)
    V, SV, SAV = keep[0]["V"], keep[0]["SV"], keep[0]["SAV"]
    j = SAV.shape[1]
    explicit = S @ (A @ V[:, :j])
    assert np.linalg.norm(SAV - explicit) <= 1e-13 * np.linalg.norm(explicit)
    np.testing.assert_allclose(SV, S @ V, atol=1e-14)


def test_sketched_residual_nonincreasing_within_cycle():
    """sres is minimised over nested spaces span([U, V(:,1:j)]) (eq. (3.2))."""
    A = _small_cd(16)
    b = randn(A.shape[0], 3)
    res = sdr_solve(A, b, m=40, k=8, t=2, s=112, tol=1e-12, max_cycles=4)
    for c in res.trace:
        h = np.array(c.sres_hist)
        assert np.all(np.diff(h) <= 1e-12 * h[0])


# -------------------------------------------------- S = I reduces to GMRES --
def _krylov_argmin(A, r0, m, U=None):
    """Dense minimum-residual correction over span([U, K_m(A, r0)])."""
    K = np.empty((r0.shape[0], m), dtype=r0.dtype)
    K[:, 0] = r0 / np.linalg.norm(r0)
    for i in range(1, m):  # orthonormalise as we go to keep K well conditioned
        w = A @ K[:, i - 1]
        for _ in range(2):
            w = w - K[:, :i] @ (K[:, :i].conj().T @ w)
        K[:, i] = w / np.linalg.norm(w)
    B = K if U is None else np.concatenate([U, K], axis=1)
    y, *_ = np.linalg.lstsq(A @ B, r0, rcond=None)
    return B @ y, B


def _dense_harmonic_ritz(A, B, k):
    """Harmonic Ritz vectors of A on range(B): (AB)^*(AB y - theta B y) = 0,
    solved without squaring as R y = theta Q^* B y with AB = QR, keeping the
    k smallest |theta| (never splitting a conjugate pair)."""
    Qa, Ra = np.linalg.qr(A @ B)
    th, Y = sla.eig(Ra, Qa.conj().T @ B)
    order = np.argsort(np.abs(th), kind="stable")
    sel = list(order[:k])
    nxt = order[k] if k < len(order) else None
    if nxt is not None and abs(th[sel[-1]].imag) > 1e-10 * abs(th[sel[-1]]) and \
            abs(th[nxt] - np.conj(th[sel[-1]])) < 1e-8 * abs(th[nxt]):
        sel.append(nxt)
    Z = B @ Y[:, sel]
    gap = abs(th[order[len(sel)]]) / abs(th[sel[-1]]) if len(sel) < len(order) else np.inf
    return Z, gap


def test_identity_sketch_full_orthogonalisation_is_gmres_dr():
    """S = I and t = m: the cycle's correction is the dense minimum-residual
    correction over span([U, K_m(A, r0)]) (Sections 2.1-2.2), the recycle space
    is spanned by dense harmonic Ritz vectors (Section 3.5 with S = I), and
    the true residual never increases from one cycle to the next, as for
    GMRES-DR (Section 2.3)."""
    N, m, k = 60, 10, 3
    A = _random_nonsym(N, 11, shift=1.5)
    b = np.random.default_rng(12).standard_normal(N)
    S = sp.identity(N, format="csr")
    keep = []
    res = sdr_solve(A, b, m=m, k=k, t=m, s=N, tol=1e-15, max_cycles=4, S=S,
                    keep_cycles=keep)
    # cycle 1: plain GMRES(m)
    xt1, B1 = _krylov_argmin(A, b, m)
    np.testing.assert_allclose(keep[0]["xt"], xt1, rtol=0, atol=1e-11 * np.linalg.norm(xt1))
    # harmonic Ritz vectors on the cycle's own search space (the Krylov space
    # itself is only determined to ~1e-8 here, the extraction much better)
    V1 = keep[0]["V"][:, :m]
    assert _max_sin_angle(V1, B1) < 1e-6
    Z, gap = _dense_harmonic_ritz(A, V1, k)
    assert gap > 1.05
    assert _max_sin_angle(keep[0]["U"], Z.real if np.isrealobj(A) and np.allclose(Z.imag, 0) else
                          np.concatenate([Z.real, Z.imag], axis=1)) < 1e-9
    # cycle 2: augmented minimum residual over span([U, K_m(A, r1)])
    r1 = keep[1]["r0"]
    U1 = keep[0]["U"]
    xt2, _ = _krylov_argmin(A, r1, m, U=U1)
    np.testing.assert_allclose(keep[1]["xt"], xt2, rtol=0, atol=1e-10 * np.linalg.norm(xt2))
    # recycle space after cycle 2: harmonic Ritz vectors on span([U1, V2])
    W2 = np.concatenate([U1, keep[1]["V"][:, :m]], axis=1)
    Z2, gap2 = _dense_harmonic_ritz(A, W2, k)
    assert gap2 > 1.05
    Z2r = np.concatenate([Z2.real, Z2.imag], axis=1)
    assert _max_sin_angle(keep[1]["U"], Z2r) < 1e-8
    r = [c.res for c in res.trace]
    assert all(r[i + 1] <= r[i] * (1 + 1e-12) for i in range(len(r) - 1))


# ------------------------------------------------- exact small eigenspace --
def _matrix_with_eigenspace(N, lam, seed, spread=0.3):
    """A = Q blkdiag(diag(lam), B) Q^{-1}: invariant subspace X = Q(:, :k) with
    eigenvalues lam, bulk B = 2I + random of radius ~spread."""
    g = np.random.default_rng(seed)
    k = len(lam)
    Q = np.eye(N) + 0.1 * g.standard_normal((N, N)) / np.sqrt(N)
    B = 2.0 * np.eye(N - k) + spread * g.standard_normal((N - k, N - k)) / np.sqrt(N)
    D = np.zeros((N, N))
    D[:k, :k] = np.diag(lam)
    D[k:, k:] = B
    A = Q @ D @ np.linalg.inv(Q)
    return A, Q[:, :k]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_exact_eigenspace_is_recovered_for_any_sketch(seed):
    """If A z = theta z with z in the search space then S(Az - theta z) = 0, so
    the sketched harmonic Ritz pair is exact for any S (Section 3.5); the
    recycle space then equals the small invariant subspace."""
    N, k = 200, 4
    lam = np.array([0.01, 0.02, 0.03, 0.04])
    A, X = _matrix_with_eigenspace(N, lam, seed)
    g = np.random.default_rng(100 + seed)
    W = _orth(np.concatenate([X, g.standard_normal((N, 16))], axis=1))
    s = 80
    S = sketch_operator(N, s, 8, 1000 + seed)
    G, ell, keff = harmonic_ritz_update(W, S @ W, S @ (A @ W), k, True, s)
    assert keff == k and ell == W.shape[1]
    assert _max_sin_angle(W @ G, X) < 1e-10


def test_exact_eigenspace_complex():
    """Complex version of the exact-eigenpair property (Section 3.5)."""
    N, k = 160, 3
    g = np.random.default_rng(7)
    Q = np.eye(N) + 0.1 * (g.standard_normal((N, N)) + 1j * g.standard_normal((N, N))) / np.sqrt(N)
    D = np.diag(np.concatenate([[0.01j, 0.02, 0.03 - 0.01j],
                                2.0 + 0.3 * (g.standard_normal(N - k) + 1j * g.standard_normal(N - k))]))
    A = Q @ D @ np.linalg.inv(Q)
    X = Q[:, :k]
    W = _orth(np.concatenate([X, g.standard_normal((N, 12)) + 1j * g.standard_normal((N, 12))], axis=1))
    s = 64
    S = sketch_operator(N, s, 8, 77)
    G, ell, keff = harmonic_ritz_update(W, S @ W, S @ (A @ W), k, False, s)
    assert keff == k
    assert _max_sin_angle(W @ G, X) < 1e-10


def test_recycled_exact_solution_space_converges_in_one_step():
    """U spanning an invariant subspace that contains A^{-1} b: the sketched
    least-squares problem is solved exactly at j = 1 (Section 3.6 reuse)."""
    N, k = 150, 4
    A, X = _matrix_with_eigenspace(N, np.array([0.1, 0.2, 0.3, 0.4]), 5)
    b = A @ (X @ np.array([1.0, -2.0, 0.5, 3.0]))
    s = 64
    S = sketch_operator(N, s, 8, 9)
    U = _orth(X)
    rec = Recycle(U, S @ U, S @ (A @ U))
    res = sdr_solve(A, b, m=20, k=k, t=2, s=s, tol=1e-10, S=S, recycle=rec)
    assert res.converged and res.cycles == 1 and res.trace[0].j_stop == 1
    x_ref = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


# ------------------------------------------------------ dense LU, chains --
@pytest.mark.parametrize("kind", ["cd", "random", "helmholtz"])
def test_solution_matches_dense_lu(kind):
    """Final x versus an LU solve: relres <= tol and forward error within
    cond(A) * tol."""
    if kind == "cd":
        A = _small_cd(12)
        b = randn(A.shape[0], 4)
    elif kind == "random":
        A = sp.csr_matrix(_random_nonsym(200, 21, shift=2.0))
        b = randn(200, 5)
    else:
        A = helmholtz2d(12, kappa=8.0).to_scipy()
        b = crandn(A.shape[0], 6)
    Ad = A.toarray()
    tol = 1e-10
    res = sdr_solve(A, b, m=20, k=5, t=2, s=64, tol=tol)
    x_ref = np.linalg.solve(Ad, b)
    assert res.converged
    assert np.linalg.norm(b - Ad @ res.x) <= tol * np.linalg.norm(b)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(res.x - x_ref) <= kappa * tol * np.linalg.norm(x_ref)


def test_residual_chain_with_exact_epsilon():
    """||r|| <= ||r~|| <= ||S r~||/sqrt(1-eps) <= ||S r||/sqrt(1-eps)
    <= sqrt((1+eps)/(1-eps)) ||r|| (eq. (3.5)) with eps the exact distortion
    of S on span([r0, A W])."""
    A = _small_cd(16)
    N = A.shape[0]
    b = randn(N, 8)
    s = 160
    S = sketch_operator(N, s, 8, 42)
    keep = []
    sdr_solve(A, b, m=12, k=4, t=2, s=s, tol=1e-14, max_cycles=2, S=S, keep_cycles=keep)
    for kc in keep:
        r0, xt = kc["r0"], kc["xt"]
        W = np.concatenate([kc["U_in"], kc["V"][:, : kc["j"]]], axis=1)
        Q = _orth(np.concatenate([r0[:, None], A @ W], axis=1))
        sv = np.linalg.svd(S @ Q, compute_uv=False)
        eps = max(sv[0] ** 2 - 1, 1 - sv[-1] ** 2)
        assert eps < 1
        y, *_ = np.linalg.lstsq(A @ W, r0, rcond=None)
        r = r0 - A @ (W @ y)
        rt = r0 - A @ xt
        c = 1 / np.sqrt(1 - eps)
        tiny = 1e-12 * np.linalg.norm(r0)
        assert np.linalg.norm(r) <= np.linalg.norm(rt) + tiny
        assert np.linalg.norm(rt) <= c * np.linalg.norm(S @ rt) + tiny
        assert np.linalg.norm(S @ rt) <= np.linalg.norm(S @ r) + tiny
        assert c * np.linalg.norm(S @ r) <= np.sqrt((1 + eps) / (1 - eps)) * np.linalg.norm(r) + tiny


def test_sketched_projector_is_idempotent():
    """The sketched residual projector Phi^ = A W (S A W)^+ S is an oblique
    projector and the cycle residual is (I - Phi^) r0 (Section 4.1)."""
    A = _small_cd(10)
    N = A.shape[0]
    b = randn(N, 9)
    S = sketch_operator(N, 64, 8, 3)
    keep = []
    sdr_solve(A, b, m=10, k=3, t=2, s=64, tol=1e-14, max_cycles=2, S=S, keep_cycles=keep)
    kc = keep[1]
    W = np.concatenate([kc["U_in"], kc["V"][:, : kc["j"]]], axis=1)
    AW = A @ W
    Phi = AW @ np.linalg.pinv((S @ AW)) @ S.toarray()
    assert np.linalg.norm(Phi @ Phi - Phi) <= 1e-9 * np.linalg.norm(Phi)
    rt = kc["r0"] - A @ kc["xt"]
    np.testing.assert_allclose(rt, kc["r0"] - Phi @ kc["r0"], atol=1e-9 * np.linalg.norm(kc["r0"]))


def test_safety_factor_update_rule():
    """A true-residual check is made only when sres < tol/safety (or at j = m);
    after a failed check the safety factor becomes res/sres (Section 3.4); every
    cycle starts at the initial 1.4."""
    A = _small_cd(32)
    b = randn(A.shape[0], 5)
    m = 50
    r = sdr_solve(A, b, m=m, k=10, t=2, s=120, tol=1e-8)
    tol_abs = 1e-8 * np.linalg.norm(b)
    assert any(len(c.checks) > 1 for c in r.trace)
    for c in r.trace:
        assert c.checks[0].safety == 1.4
        for ch in c.checks:
            assert ch.sres < tol_abs / ch.safety or ch.j == m
        for prev, nxt in zip(c.checks[:-1], c.checks[1:]):
            assert prev.res >= tol_abs
            assert nxt.safety == prev.res / prev.sres


# -------------------------------------------------------------- sequences --
def test_sequence_exact_and_inexact_sau():
    """Section 3.6: the exact variant recomputes S A^(i+1) U, the inexact one
    keeps S A^(i) U; recycling reduces the work of the next system."""
    A1c = cd2d_upwind(16)
    A1 = A1c.to_scipy()
    N = A1.shape[0]
    d = 0.05 * np.random.default_rng(3).uniform(0, 1, N)
    A2 = shifted_diagonal(A1c, d).to_scipy()
    b1, b2 = randn(N, 1), randn(N, 2)
    kw = dict(m=30, k=8, t=2, s=80, tol=1e-10)
    S = sketch_operator(N, 80, 8, 42)
    r1 = sdr_solve(A1, b1, S=S, **kw)
    keep = []
    r2 = sdr_solve(A2, b2, S=S, recycle=r1.recycle, new_matrix=True, keep_cycles=keep, **kw)
    U = r1.recycle.U
    np.testing.assert_allclose(keep[0]["SAU_in"], S @ (A2 @ U), atol=1e-12)
    np.testing.assert_allclose(keep[0]["SU_in"], S @ U, atol=1e-12)
    keep_in = []
    sdr_solve(A2, b2, S=S, recycle=r1.recycle, new_matrix=True, variant="inexact",
              keep_cycles=keep_in, max_cycles=1, **kw)
    np.testing.assert_allclose(keep_in[0]["SAU_in"], S @ (A1 @ U), atol=1e-12)
    assert r2.converged
    # recycling pays where a few small eigenvalues are isolated from the bulk
    # (the situation of the paper's sequence experiments): U carried to a
    # slightly changed matrix cuts the Arnoldi steps well below a cold start
    N = 400
    B1, _ = _matrix_with_eigenspace(N, np.array([1e-3, 2e-3, 3e-3, 4e-3]), 4, spread=1.0)
    g = np.random.default_rng(0)
    B2 = B1 + np.diag(1e-4 * g.uniform(0, 1, N))
    c1, c2 = g.standard_normal(N), g.standard_normal(N)
    kw = dict(m=20, k=4, t=2, s=48, tol=1e-10)
    w1 = sdr_solve(B1, c1, **kw)
    w2 = sdr_solve(B2, c2, recycle=w1.recycle, new_matrix=True, **kw)
    cold = sdr_solve(B2, c2, **kw)
    assert w2.converged and cold.converged
    assert w2.iters < 0.7 * cold.iters


def test_real_problem_as_complex_gives_real_result():
    """A real system cast to complex128 follows the same first cycle, with the
    conjugation convention H(i,j) = V(:,i)^* w (Algorithm 1)."""
    A = _small_cd(12)
    b = randn(A.shape[0], 4)
    kw = dict(m=20, k=5, t=2, s=64, tol=1e-14, max_cycles=1)
    rr = sdr_solve(A, b, **kw)
    rc = sdr_solve(A.astype(np.complex128), b.astype(np.complex128), **kw)
    np.testing.assert_allclose(rc.x.real, rr.x, atol=1e-12 * np.linalg.norm(rr.x))
    assert np.linalg.norm(rc.x.imag) <= 1e-12 * np.linalg.norm(rr.x)
    Uc, Ur = rc.recycle.U, rr.recycle.U
    # complex selection is contained in the (pair-closed) real selection
    resid = Uc - Ur @ np.linalg.lstsq(Ur, Uc, rcond=None)[0]
    assert np.linalg.norm(resid) <= 1e-9 * np.linalg.norm(Uc)


# ------------------------------------------------------------ failure modes --
def test_not_converged_and_breakdown_paths():
    A = _small_cd(16)
    b = randn(A.shape[0], 1)
    r = sdr_solve(A, b, m=5, k=2, t=2, s=32, tol=1e-12, max_cycles=1)
    assert not r.converged and r.cycles == 1 and r.relres > 1e-12
    # singular: b not in range(A), A b = 0 -> breakdown at j = 1
    N = 30
    D = sp.diags(np.concatenate([[0.0], np.arange(1.0, N)])).tocsr()
    e0 = np.zeros(N)
    e0[0] = 1.0
    r = sdr_solve(D, e0, m=5, k=2, t=2, s=16, tol=1e-10, max_cycles=3)
    assert not r.converged
    assert r.trace[0].breakdown and r.trace[0].j_stop == 1
    # happy breakdown on an invariant Krylov space: exact solution
    Dd = sp.diags(np.arange(1.0, N + 1)).tocsr()
    bb = np.zeros(N)
    bb[:3] = 1.0
    Dd = sp.diags(np.concatenate([[1.0, 2.0, 3.0], 5.0 * np.ones(N - 3)])).tocsr()
    bb = np.ones(N)
    r = sdr_solve(Dd, bb, m=10, k=2, t=3, s=32, tol=1e-12)
    assert r.converged and r.trace[0].j_stop <= 4


def test_rank_loss_leaves_the_dependent_column_out():
    """A cycle that stops because SAW loses rank (the paper is silent; the
    oracle's reading): the stop is the first step whose new SAW column lies
    within rank_rtol (relative) of the span of the earlier columns, measured
    here by a Householder QR of those columns; the column adds no direction,
    so the sketched residual at the stop is the minimum over the earlier
    columns (projection with the same QR) and the column's coefficient is 0.
    Window t = 1 makes SAW nearly dependent within 40 steps."""
    A = cd2d_upwind(23)
    b = randn(A.n, 23)
    keep = []
    r = sdr_solve(A.to_scipy(), b, m=40, k=8, t=1, s=104, tol=1e-9, rank_rtol=1e-4,
                  max_cycles=1, keep_cycles=keep)
    c = r.trace[0]
    assert c.rank_loss and c.j_stop == len(c.sres_hist)
    kp = keep[0]
    SAV, j, Sr = kp["SAV"], kp["j"], kp["Sr"]
    dist = []
    for jj in range(2, j + 1):
        Q, _ = np.linalg.qr(SAV[:, : jj - 1])
        a = SAV[:, jj - 1]
        dist.append(np.linalg.norm(a - Q @ (Q.T @ a)) / np.linalg.norm(a))
    assert dist[-1] <= 1e-4 < min(dist[:-1])
    Q, _ = np.linalg.qr(SAV[:, : j - 1])
    smin = np.linalg.norm(Sr - Q @ (Q.T @ Sr))
    # (SAW is ill-conditioned here: lstsq and this QR agree to ~1e-12)
    assert abs(c.sres - smin) <= 1e-9 * smin
    assert c.sres_hist[-1] == c.sres_hist[-2]
    assert kp["y"][-1] == 0.0
    # and the true residual of the check is that of the returned iterate
    assert abs(c.res - np.linalg.norm(b - A.to_scipy() @ r.x)) <= 1e-12 * np.linalg.norm(b)
