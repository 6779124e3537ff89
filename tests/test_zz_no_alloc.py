"""The allocation-free sketch entry point against sdr_sketch.

sdr_sketch_noalloc keeps its partial sums in a static device array instead
of a handle's buffers; its output must equal what sdr_sketch gives on a
handle drawn from the same seed, s_dim and zeta (the same kernels, so the
same bits are expected; the bar is 1e-14 relative), and the oracle's S X to
1e-12.  Two calls in a row, the second on a smaller input, check that the
scratch's leftover contents from the first never leak into the second.
"""

import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.sketch import sketch_operator
from workloads import CSR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _handle_sketch(N, s, zeta, seed, X):
    from paper_2311_14206_amd.sdr import SDRSolver
    # a handle of X's data type (the matrix itself plays no part in S X)
    A = CSR.from_scipy(sp.identity(N, dtype=X.cpu().numpy().dtype, format="csr"))
    h = SDRSolver(torch.from_numpy(A.row_ptr).to(DEV), torch.from_numpy(A.col_idx).to(DEV),
                  torch.from_numpy(A.values).to(DEV), m=8, k=2, t=2, s=s, seed=seed, zeta=zeta)
    Y = h.sketch(X).cpu().numpy()
    h.close()
    return Y


def _case(N, s, zeta, seed, cols, cpx, rng):
    from paper_2311_14206_amd.sdr import sketch_noalloc
    print(f"[gpu] sketch_noalloc N={N} s={s} zeta={zeta} cols={cols} complex={cpx}", flush=True)
    X = rng.standard_normal((N, cols))
    if cpx:
        X = X + 1j * rng.standard_normal((N, cols))
    Xd = torch.from_numpy(X).to(DEV)
    Y = sketch_noalloc(Xd, s, seed=seed, zeta=zeta)
    torch.cuda.synchronize()
    Y = Y.cpu().numpy()
    ref = _handle_sketch(N, s, zeta, seed, Xd)
    same = np.array_equal(Y, ref)
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    print(f"[gpu]   vs sdr_sketch: bit-identical {same}, rel. diff {err:.1e}", flush=True)
    assert err <= 1e-14
    So = sketch_operator(N, s, zeta, seed)
    ora = So @ X
    assert np.linalg.norm(Y - ora) <= 1e-12 * np.linalg.norm(ora)


@pytest.mark.parametrize("cpx", [False, True])
def test_noalloc_sketch_matches_sdr_sketch_two_calls(cpx):
    rng = np.random.default_rng(2024 + cpx)
    # first call: many tiles, a ragged tail, more columns than one launch takes
    _case(300_001, 240, 8, 42, 11, cpx, rng)
    # second call, smaller: another seed and zeta, fewer rows and columns
    _case(5_003, 120, 6, 7, 3, cpx, rng)


def test_noalloc_sketch_single_vector_and_errors():
    from paper_2311_14206_amd.sdr import sketch_noalloc, lib, SDRError
    rng = np.random.default_rng(9)
    x = rng.standard_normal(4096)
    xd = torch.from_numpy(x).to(DEV)
    y = sketch_noalloc(xd, 64, seed=3, zeta=8)
    torch.cuda.synchronize()
    ora = sketch_operator(4096, 64, 8, 3) @ x
    assert np.linalg.norm(y.cpu().numpy() - ora) <= 1e-12 * np.linalg.norm(ora)
    with pytest.raises(SDRError, match="multiple of zeta"):
        sketch_noalloc(xd, 60, seed=3, zeta=8)
    # beyond the scratch: rejected before any device work
    rc = lib().sdr_sketch_noalloc(1 << 30, 2048, 8, 1, 0, C.c_void_p(xd.data_ptr()), 1,
                                  C.c_void_p(xd.data_ptr()), None)
    assert rc == -1 and b"scratch" in lib().sdr_last_error()
