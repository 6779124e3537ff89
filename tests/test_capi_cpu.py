"""C interface checks that need no GPU: the library loads, exports every
function declared in include/sdr.h, and its host-side harmonic-Ritz step
agrees with the oracle's ordered-QZ route (Section 3.5)."""

import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2311_14206_amd", "libsdr.so")
HDR = os.path.join(ROOT, "include", "sdr.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsdr.so not built")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdr_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    names = _declared()
    assert "sdr_create" in names and "sdr_solve" in names and "sdr_update_matrix" in names
    for n in names:
        assert hasattr(L, n), n


def _orth(X):
    return sla.orth(X)


def _angle(X, Y):
    Qx, Qy = _orth(X), _orth(Y)
    return max(np.linalg.norm(Qy - Qx @ (Qx.conj().T @ Qy), 2),
               np.linalg.norm(Qx - Qy @ (Qy.conj().T @ Qx), 2))


def _case(seed, s, l0, cplx, rank_def=False):
    g = np.random.default_rng(seed)
    if cplx:
        SAW = g.standard_normal((s, l0)) + 1j * g.standard_normal((s, l0))
        SB = g.standard_normal((s, l0)) + 1j * g.standard_normal((s, l0))
    else:
        SAW = g.standard_normal((s, l0))
        SB = g.standard_normal((s, l0))
    if rank_def:
        SAW[:, -1] = SAW[:, 0] + 1e-15 * SAW[:, 1]
    return SAW, SB


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_host_harmonic_ritz_matches_oracle(cplx, seed):
    from oracle import harmonic_ritz_update
    from paper_2311_14206_amd.sdr import host_harmonic_ritz
    s, l0, k = 96, 40, 8
    SAW, SB = _case(seed, s, l0, cplx)
    Q, R = np.linalg.qr(SAW)
    Cm = Q.conj().T @ SB
    G, ell, keff = host_harmonic_ritz(R, Cm, s, k, cplx)
    Go, ello, keffo = harmonic_ritz_update(np.eye(l0), SB, SAW, k, not cplx, s)
    assert keff == keffo and ell == ello
    assert _angle(G, Go) < 1e-9
    if not cplx:
        assert np.isrealobj(G)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("seed", [3, 4])
def test_host_harmonic_ritz_matches_oracle_full_size(cplx, seed):
    """The cycle's size of the timed workload: ell0 = k + m = 120, s = 240."""
    from oracle import harmonic_ritz_update
    from paper_2311_14206_amd.sdr import host_harmonic_ritz
    s, l0, k = 240, 120, 20
    SAW, SB = _case(seed, s, l0, cplx)
    Q, R = np.linalg.qr(SAW)
    G, ell, keff = host_harmonic_ritz(R, Q.conj().T @ SB, s, k, cplx)
    Go, ello, keffo = harmonic_ritz_update(np.eye(l0), SB, SAW, k, not cplx, s)
    assert keff == keffo and ell == ello
    assert _angle(G, Go) < 1e-8
    assert np.linalg.norm(G.conj().T @ G - np.eye(keff)) < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_host_harmonic_ritz_truncated_svd_path(cplx):
    """A numerically dependent column of SAW: the truncated SVD drops it."""
    from oracle import harmonic_ritz_update
    from paper_2311_14206_amd.sdr import host_harmonic_ritz
    s, l0, k = 64, 20, 5
    SAW, SB = _case(7, s, l0, cplx, rank_def=True)
    Q, R = np.linalg.qr(SAW)
    G, ell, keff = host_harmonic_ritz(R, Q.conj().T @ SB, s, k, cplx)
    Go, ello, keffo = harmonic_ritz_update(np.eye(l0), SB, SAW, k, not cplx, s)
    assert ell == ello == l0 - 1
    assert keff == keffo
    assert _angle(G, Go) < 1e-7


def test_noalloc_sketch_rejects_sizes_beyond_its_scratch():
    """The allocation-free sketch checks its limits before touching a device."""
    L = ctypes.CDLL(LIB)
    f = L.sdr_sketch_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.sdr_last_error.restype = ctypes.c_char_p
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
    assert f(1 << 28, 240, 8, 1, 0, fake, 1, fake, None) == -1
    assert b"scratch" in L.sdr_last_error()
    assert f(1000, 100, 8, 1, 0, fake, 1, fake, None) == -1  # s_dim not a multiple of zeta
    assert f(1000, 4096, 8, 1, 0, fake, 1, fake, None) == -1  # s_dim beyond the LDS bins
    assert f(1000, 2048, 8, 1, 2, fake, 1, fake, None) == -1  # complex beyond 1024
    assert f(1000, 240, 8, 1, 1, fake, 1, fake, None) == -1  # FP32 is not a data type here
    assert f(0, 240, 8, 1, 0, fake, 1, fake, None) == -1


@pytest.mark.parametrize("seed", [5, 6])
def test_host_harmonic_ritz_complex_helmholtz_shape(seed):
    """The size of the complex Helmholtz cycle: ell0 = k + m = 180, s = 360,
    k = 30 (random data, whose selected eigenvalues need not lead the Schur
    form)."""
    from oracle import harmonic_ritz_update
    from paper_2311_14206_amd.sdr import host_harmonic_ritz
    s, l0, k = 360, 180, 30
    SAW, SB = _case(seed, s, l0, True)
    Q, R = np.linalg.qr(SAW)
    G, ell, keff = host_harmonic_ritz(R, Q.conj().T @ SB, s, k, True)
    Go, ello, keffo = harmonic_ritz_update(np.eye(l0), SB, SAW, k, False, s)
    assert keff == keffo == k and ell == ello
    assert _angle(G, Go) < 1e-8
    assert np.linalg.norm(G.conj().T @ G - np.eye(keff)) < 1e-12


def test_host_harmonic_ritz_on_helmholtz_cycles():
    """Two cycles of a complex shifted Helmholtz solve with the full-size
    m = 150, k = 30, t = 3, s = 360 (the second has ell0 = 180): the library's
    step spans the oracle's recycle space, to within the first-order
    perturbation bound of an invariant subspace, eps cond(R) / (relative gap
    between the k-th and (k+1)-th largest |mu|), with a factor 100."""
    from oracle import sdr_solve
    from paper_2311_14206_amd.sdr import host_harmonic_ritz
    from workloads import helmholtz2d, crandn
    A = helmholtz2d(96, kappa=40.0).to_scipy()
    b = crandn(A.shape[0], 3)
    keep = []
    sdr_solve(A, b, m=150, k=30, t=3, s=360, tol=1e-14, max_cycles=2, keep_cycles=keep)
    assert keep[1]["j"] + keep[1]["U_in"].shape[1] == 180
    for kc in keep:
        j = kc["j"]
        SAW = np.concatenate([kc["SAU_in"], kc["SAV"][:, :j]], axis=1)
        SB = np.concatenate([kc["SU_in"], kc["SV"][:, :j]], axis=1)
        Q, R = np.linalg.qr(SAW)
        Cm = Q.conj().T @ SB
        G, ell, keff = host_harmonic_ritz(R, Cm, 360, 30, True)
        assert keff == kc["G"].shape[1]
        mu = np.sort(np.abs(np.linalg.eigvals(np.linalg.solve(R, Cm))))[::-1]
        bound = 100 * 2.0 ** -52 * np.linalg.cond(R) / ((mu[29] - mu[30]) / mu[29])
        ang = _angle(G, kc["G"])
        print(f"ell0 {R.shape[0]}: angle {ang:.1e}, bound {bound:.1e}")
        assert ang < max(bound, 1e-10)
