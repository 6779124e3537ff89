"""Constant diagonals of the diagonal storage (option dia_const).

When every entry of a diagonal inside the matrix has the same bits, as in a
constant-coefficient stencil, the step kernel takes that value from its
arguments instead of reading the diagonal's stream.  The products are the
same numbers, so a solve must return the same bits with the option on and
off, and the mask must name exactly the constant diagonals.
"""

import numpy as np
import pytest

from workloads import cd2d_upwind, crandn, edge_weighted, helmholtz2d, randn, shifted_diagonal

import test_gpu_parity as gp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _constant_mask(A, offsets):
    """Host reference: bit d set when diagonal offsets[d] holds one value
    (bitwise) on every row where it lies inside the matrix."""
    dense = {}
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    for r, c, v in zip(rows, A.col_idx, A.values):
        dense[(int(r), int(c))] = v
    mask = 0
    for d, off in enumerate(offsets):
        vals = [dense.get((r, r + off), 0.0) for r in range(max(0, -off), min(A.n, A.n - off))]
        if vals and all(np.asarray(v).tobytes() == np.asarray(vals[0]).tobytes() for v in vals):
            mask |= 1 << d
    return mask


def _solve_pair(A, b, kw, tol, **opt):
    out = []
    for dc in (1, 0):
        h = gp._solver(A, dia_const=dc, **kw, **opt)
        x, st = h.solve(gp._dev(b), tol=tol)
        out.append((h, gp._host(x), st))
    return out


@pytest.mark.parametrize("case", ["cd2d", "helmholtz", "shifted", "weighted", "cd2d_fp32"])
def test_constant_diagonals_same_bits(case):
    opt = {}
    if case == "cd2d":
        A, b = cd2d_upwind(48), randn(48 * 48, 5)
    elif case == "cd2d_fp32":
        A, b = cd2d_upwind(48), randn(48 * 48, 5)
        opt = dict(precision=1)
    elif case == "helmholtz":
        A, b = helmholtz2d(40, kappa=8.0), crandn(40 * 40, 6)
    elif case == "shifted":
        A0 = cd2d_upwind(48)
        A = shifted_diagonal(A0, 1e-3 * np.random.default_rng(7).uniform(0.0, 1.0, A0.n))
        b = randn(A.n, 8)
    else:
        A0 = cd2d_upwind(48)
        A = edge_weighted(A0, 1.0 + 0.1 * randn(A0.nnz, 9))
        b = randn(A.n, 10)
    kw = dict(m=30, k=6, t=2, s=64)
    (h1, x1, st1), (h0, x0, st0) = _solve_pair(A, b, kw, 1e-9, **opt)
    offsets = h1.spmv_layout()
    assert offsets, "stencil pattern stored by diagonals"
    mask = h1.const_diagonals()
    want = _constant_mask(A, offsets)
    print(f"{case}: offsets {offsets}, constant mask {mask:#x} (host {want:#x}), "
          f"{st1['iters']} steps", flush=True)
    assert mask == want
    assert h0.const_diagonals() == 0
    n = int(round(np.sqrt(A.n)))
    if case in ("cd2d", "helmholtz", "cd2d_fp32"):
        # the main diagonal and the +-n ones; the +-1 ones hold zeros where a
        # grid line ends
        assert mask == sum(1 << offsets.index(o) for o in (-n, 0, n))
    if case == "shifted":
        assert mask == sum(1 << offsets.index(o) for o in (-n, n))
    assert st1["iters"] == st0["iters"] and st1["cycles"] == st0["cycles"]
    assert x1.tobytes() == x0.tobytes()
    assert [c["j_stop"] for c in h1.trace()] == [c["j_stop"] for c in h0.trace()]


def test_constant_diagonals_follow_matrix_updates():
    """A sequence moving from a constant-coefficient matrix to a shifted one
    and back: the mask is found again after each update."""
    A0 = cd2d_upwind(40)
    A1 = shifted_diagonal(A0, 1e-2 * np.random.default_rng(3).uniform(0.0, 1.0, A0.n))
    b = randn(A0.n, 11)
    kw = dict(m=30, k=6, t=2, s=64)
    h = gp._solver(A0, dia_const=1, **kw)
    ref = gp._solver(A0, dia_const=0, **kw)
    offsets = None
    for A in (A0, A1, A0):
        for s_ in (h, ref):
            s_.update_matrix(gp._dev(A.values))
        x, _ = h.solve(gp._dev(b), tol=1e-9)
        xr, _ = ref.solve(gp._dev(b), tol=1e-9)
        offsets = h.spmv_layout()
        assert h.const_diagonals() == _constant_mask(A, offsets)
        assert gp._host(x).tobytes() == gp._host(xr).tobytes()
