"""Pins of the oracle's subsampled randomised DCT sketch S = sqrt(N/s) P F E
(Section 6): with every row kept S = F E is orthogonal; a column of S follows
the DCT-II definition written out; the random signs and rows come from the
stated generator (checked against a big-integer transcription); S embeds a
small subspace; GMRES-SDR with this sketch reaches the dense LU solutions and
recovers exact eigenspaces as with any sketch."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import SRDCT, sdr_solve, srdct_rows, srdct_signs
from workloads import cd2d_upwind, helmholtz2d, randn, crandn

M64 = (1 << 64) - 1


def _mix64_int(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


@pytest.mark.parametrize("N", [64, 101])
def test_all_rows_kept_is_an_isometry(N):
    S = SRDCT(N, N, 9)
    M = S.toarray()
    assert np.abs(M.T @ M - np.eye(N)).max() < 1e-13
    x = randn(N, 1)
    assert abs(np.linalg.norm(S @ x) - np.linalg.norm(x)) < 1e-13 * np.linalg.norm(x)
    z = crandn(N, 2)
    assert abs(np.linalg.norm(S @ z) - np.linalg.norm(z)) < 1e-13 * np.linalg.norm(z)


def test_columns_follow_the_dct_definition():
    """S[i, n] = sqrt(N/s) c_p cos(pi p (2n + 1) / (2N)) e_n with p = rows[i],
    c_0 = sqrt(1/N), c_p = sqrt(2/N): the orthonormal DCT-II, subsampled."""
    N, s = 12, 5
    S = SRDCT(N, s, 4)
    M = S.toarray()
    e, rows = srdct_signs(N, 4), srdct_rows(N, s, 4)
    for i, p in enumerate(rows):
        c = np.sqrt(1.0 / N) if p == 0 else np.sqrt(2.0 / N)
        for n in range(N):
            ref = np.sqrt(N / s) * c * np.cos(np.pi * p * (2 * n + 1) / (2 * N)) * e[n]
            assert abs(M[i, n] - ref) < 1e-14


def test_signs_and_rows_follow_the_generator():
    """Against a transcription of the definition in Python integers."""
    N, s, seed = 300, 40, 0xDEADBEEF12345
    e = srdct_signs(N, seed)
    rows = srdct_rows(N, s, seed)
    g = 0x9E3779B97F4A7C15
    ks = [_mix64_int(((seed ^ 0x5851F42D4C957F2D) + g * (n + 1)) & M64) for n in range(N)]
    assert np.array_equal(e, np.array([-1.0 if k & 1 else 1.0 for k in ks]))
    kr = [(_mix64_int(((seed ^ 0x14057B7EF767814F) + g * (n + 1)) & M64), n) for n in range(N)]
    ref = sorted(n for _, n in sorted(kr)[:s])
    assert rows.tolist() == ref
    assert len(set(rows.tolist())) == s and rows.min() >= 0 and rows.max() < N
    big = srdct_signs(20000, 1)
    assert abs(np.mean(big)) < 4.0 / np.sqrt(20000)  # (a fair coin: within four deviations)


def test_embeds_a_small_subspace():
    """eq. (3.1) for a 10-dimensional subspace: every singular value of S Q
    within [0.5, 1.5]; over 100 seeds the mean of ||S x||^2 / ||x||^2 is 1
    within 5% (E ||S x||^2 = ||x||^2)."""
    N, s = 2048, 256
    Q = sla.orth(np.random.default_rng(3).standard_normal((N, 10)))
    sv = np.linalg.svd(SRDCT(N, s, 11) @ Q, compute_uv=False)
    assert 0.5 < sv.min() and sv.max() < 1.5
    x = randn(N, 12)
    r = [np.linalg.norm(SRDCT(N, s, sd) @ x) ** 2 / np.linalg.norm(x) ** 2 for sd in range(100)]
    assert abs(np.mean(r) - 1.0) < 0.05


def test_srdct_solve_matches_dense_lu():
    for A, b in ((cd2d_upwind(16).to_scipy(), randn(256, 9)),
                 (helmholtz2d(12, kappa=4.0).to_scipy(), crandn(144, 9))):
        tol = 1e-10
        r = sdr_solve(A, b, m=20, k=5, t=2, s=64, tol=tol, sketch="srdct")
        assert r.converged
        Ad = A.toarray()
        x = np.linalg.solve(Ad, b)
        assert np.linalg.norm(r.x - x) <= np.linalg.cond(Ad) * tol * np.linalg.norm(x)


def test_exact_eigenspace_is_recovered_with_srdct():
    """An exact invariant subspace in the search space is a sketched harmonic
    Ritz space for any sketch (Section 3.5), this one included."""
    import scipy.sparse as sp
    N, k = 200, 3
    d = np.concatenate([[1e-3, 2e-3, 3e-3], np.linspace(1.0, 2.0, N - 3)])
    A = sp.diags(d).tocsr()
    b = randn(N, 13)
    r = sdr_solve(A, b, m=30, k=k, t=30, s=96, tol=1e-14, max_cycles=1, sketch="srdct")
    U = r.recycle.U
    E = np.zeros((N, k))
    E[:3, :] = np.eye(3)
    Qa, Qb = sla.orth(U), E
    assert np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2) < 1e-8
