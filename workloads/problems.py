"""Synthetic sparse operators and seeded vectors.

Operators (all on the unit square/cube, mesh width h = 1/(n+1), homogeneous
Dirichlet boundary eliminated, unknowns ordered lexicographically with x
fastest, every entry scaled by h^2):

* ``cd2d_upwind``  -Laplace(u) + beta . grad(u), first-order upwind convection
  (beta > 0 componentwise): diagonal 4 + h(bx+by), west -1-h*bx, south -1-h*by,
  east and north -1.  5 entries per interior row, nnz = 5n^2 - 4n.
* ``cd3d_upwind``  7-point analogue: diagonal 6 + h(bx+by+bz), west/south/down
  -1-h*b, east/north/up -1.  nnz = 7n^3 - 6n^2.
* ``helmholtz2d``  -Laplace(u) - kappa^2 (1 + 0.5i) u: diagonal
  4 - (kappa h)^2 (1+0.5i), neighbours -1 (complex128).
* ``cd2d_central`` the convection-diffusion family of the paper's last
  experiment (Section 6.3): (L (x) I + I (x) L) + alpha (D (x) I + I (x) D) with
  L = (n+1)^2 tridiag(1,-2,1) and D = (n+1)/2 tridiag(-1,0,1).
* ``theta_weighted`` scales every stored entry of a base matrix by theta_e.
* ``column_scaled`` multiplies column j of a base matrix by c_j (a badly
  scaled unknown per column; ``log_uniform`` draws such scales).
* ``edge_weighted``  weights the grid edges (off-diagonal entries) by theta_e
  and sets each diagonal so that the row keeps the base matrix's row sum: a
  weighted upwind operator that stays a nonsingular M-matrix.

These are problem inputs only: nothing here belongs to the solver.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """Compressed sparse row matrix with 32-bit indices (host arrays)."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    values: np.ndarray   # float64 / complex128 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def dtype(self):
        return self.values.dtype

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr),
                             shape=(self.n, self.n))

    def with_values(self, values: np.ndarray) -> "CSR":
        values = np.ascontiguousarray(values)
        assert values.shape == self.values.shape
        return CSR(self.n, self.row_ptr, self.col_idx, values)

    @staticmethod
    def from_scipy(a) -> "CSR":
        a = sp.csr_matrix(a)
        a.sort_indices()
        return CSR(a.shape[0], a.indptr.astype(np.int32),
                   a.indices.astype(np.int32), np.ascontiguousarray(a.data))


def _stencil(n: int, dim: int, coeffs: dict, dtype) -> CSR:
    """Assemble a constant-coefficient stencil on an n^dim grid.

    ``coeffs`` maps an offset tuple (dx, dy[, dz]) to its value.  Neighbours
    outside the grid are dropped (Dirichlet elimination).  Columns in each row
    come out sorted because offsets are visited in increasing linear offset.
    """
    N = n ** dim
    idx = np.arange(N, dtype=np.int64)
    coords = [(idx // (n ** a)) % n for a in range(dim)]  # x fastest
    strides = [n ** a for a in range(dim)]
    offs = sorted(coeffs.keys(), key=lambda o: sum(o[a] * strides[a] for a in range(dim)))
    cols_per_off, vals_per_off, masks = [], [], []
    for o in offs:
        mask = np.ones(N, dtype=bool)
        for a in range(dim):
            if o[a] != 0:
                c = coords[a] + o[a]
                mask &= (c >= 0) & (c < n)
        lin = sum(o[a] * strides[a] for a in range(dim))
        masks.append(mask)
        cols_per_off.append(idx + lin)
        vals_per_off.append(coeffs[o])
    mask_mat = np.stack(masks, axis=1)                # N x n_off
    col_mat = np.stack(cols_per_off, axis=1)
    val_mat = np.broadcast_to(np.array(vals_per_off, dtype=dtype), mask_mat.shape)
    counts = mask_mat.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = col_mat[mask_mat].astype(np.int32)      # row-major => sorted per row
    values = np.ascontiguousarray(val_mat[mask_mat]).astype(dtype)
    return CSR(N, row_ptr.astype(np.int32), col_idx, values)


def cd2d_upwind(n: int, beta=(50.0, 50.0)) -> CSR:
    h = 1.0 / (n + 1)
    bx, by = beta
    c = {(0, 0): 4.0 + h * (bx + by),
         (-1, 0): -1.0 - h * bx, (1, 0): -1.0,
         (0, -1): -1.0 - h * by, (0, 1): -1.0}
    return _stencil(n, 2, c, np.float64)


def cd3d_upwind(n: int, beta=(50.0, 50.0, 50.0)) -> CSR:
    h = 1.0 / (n + 1)
    bx, by, bz = beta
    c = {(0, 0, 0): 6.0 + h * (bx + by + bz),
         (-1, 0, 0): -1.0 - h * bx, (1, 0, 0): -1.0,
         (0, -1, 0): -1.0 - h * by, (0, 1, 0): -1.0,
         (0, 0, -1): -1.0 - h * bz, (0, 0, 1): -1.0}
    return _stencil(n, 3, c, np.float64)


def helmholtz2d(n: int, kappa: float = 20.0, damping: float = 0.5) -> CSR:
    h = 1.0 / (n + 1)
    d = 4.0 - (kappa * h) ** 2 * (1.0 + 1j * damping)
    c = {(0, 0): d, (-1, 0): -1.0, (1, 0): -1.0, (0, -1): -1.0, (0, 1): -1.0}
    return _stencil(n, 2, c, np.complex128)


def cd2d_central(n: int, alpha: float) -> CSR:
    """Section 6.3 operator (central differences, unscaled)."""
    s2 = float(n + 1) ** 2
    s1 = (n + 1) / 2.0
    # L (x) I + I (x) L contributes s2*(-4) on the diagonal and s2 off-diagonal.
    # D (x) I + I (x) D: D = s1*tridiag(-1, 0, 1): +s1 east/north, -s1 west/south.
    c = {(0, 0): -4.0 * s2,
         (-1, 0): s2 - alpha * s1, (1, 0): s2 + alpha * s1,
         (0, -1): s2 - alpha * s1, (0, 1): s2 + alpha * s1}
    return _stencil(n, 2, c, np.float64)


def theta_weighted(base: CSR, theta: np.ndarray) -> CSR:
    """Entrywise reweighting vals(theta) = theta * vals(base)."""
    theta = np.asarray(theta)
    assert theta.shape == base.values.shape
    return base.with_values(theta * base.values)


def _diag_positions(base: CSR):
    rows = np.repeat(np.arange(base.n), np.diff(base.row_ptr))
    return rows, rows == base.col_idx


def edge_weighted(base: CSR, theta: np.ndarray) -> CSR:
    """Off-diagonal entries theta_e * a_e; diagonal a_ii + sum_j (1 - theta_ij) a_ij.

    theta has one entry per stored entry; the diagonal ones are unused.
    """
    theta = np.asarray(theta, dtype=np.float64)
    rows, on = _diag_positions(base)
    off = ~on
    vals = base.values.copy()
    vals[off] = theta[off] * base.values[off]
    shift = np.zeros(base.n, dtype=base.values.dtype)
    np.add.at(shift, rows[off], (1.0 - theta[off]) * base.values[off])
    vals[on] = base.values[on] + shift[rows[on]]
    return base.with_values(vals)


def shifted_diagonal(base: CSR, d: np.ndarray) -> CSR:
    """base + diag(d) on the same pattern (every row holds its diagonal)."""
    rows = np.repeat(np.arange(base.n), np.diff(base.row_ptr))
    diag_pos = np.nonzero(base.col_idx == rows)[0]
    assert diag_pos.shape[0] == base.n, "pattern must hold every diagonal entry"
    vals = base.values.copy()
    vals[diag_pos] += d
    return base.with_values(vals)


def column_scaled(base: CSR, c: np.ndarray) -> CSR:
    """base diag(c): every stored entry (i, j) multiplied by c_j."""
    c = np.asarray(c)
    assert c.shape == (base.n,)
    return base.with_values(base.values * c[base.col_idx])


def log_uniform(n: int, lo: float, hi: float, seed: int, pow2: bool = False) -> np.ndarray:
    """n values 10^U(lo, hi) (PCG64); with pow2, the nearest powers of two."""
    e = np.random.default_rng(seed).uniform(lo, hi, n)
    if pow2:
        return np.exp2(np.round(e * np.log2(10.0)))
    return 10.0 ** e


def randn(n: int, seed: int) -> np.ndarray:
    """N(0,1) vector from NumPy's PCG64 generator."""
    return np.random.default_rng(seed).standard_normal(n)


def crandn(n: int, seed: int) -> np.ndarray:
    """CN(0,1): real and imaginary parts N(0,1/2), real part drawn first."""
    g = np.random.default_rng(seed)
    re = g.standard_normal(n)
    im = g.standard_normal(n)
    return np.sqrt(0.5) * (re + 1j * im)


# ---------------------------------------------------------------------------
# Named workloads: operator sizes and method parameters.
# ---------------------------------------------------------------------------
WORKLOADS = {
    # 2D upwind convection-diffusion 64^2, Peclet 50, real FP64.
    "cd2d_64": dict(kind="cd2d_upwind", n=64, m=50, k=10, t=2, s=120, zeta=8,
                    tol=1e-8, b_seed=1, s_seed=42),
    # same operator, 1024^2 (N = 1,048,576).
    "cd2d_1024": dict(kind="cd2d_upwind", n=1024, m=100, k=20, t=2, s=240, zeta=8,
                      tol=1e-8, b_seed=1, s_seed=42),
    # 3D upwind convection-diffusion 128^3, 20 diagonally shifted systems.
    "cd3d_128_seq": dict(kind="cd3d_upwind", n=128, m=100, k=20, t=2, s=240, zeta=8,
                         tol=1e-8, n_systems=20, d_scale=1e-3, d_seed0=100,
                         b_seed0=200, s_seed=42),
    # complex shifted Helmholtz 1024^2.
    "helmholtz_1024": dict(kind="helmholtz2d", n=1024, kappa=20.0, m=150, k=30, t=3,
                           s=360, zeta=8, tol=1e-8, b_seed=3, s_seed=42),
    # theta-weighted convection-diffusion 512^2 for the differentiated solve.
    "cd2d_512_theta": dict(kind="cd2d_upwind", n=512, m=100, k=20, t=2, s=240, zeta=8,
                           tol=1e-8, theta_seed=7, xt_seed=8, b_seed=9, fd_seed=10,
                           gd_steps=50, s_seed=42),
}


def describe(name: str) -> str:
    """One-line description of a named workload (operator, size, inputs)."""
    p = WORKLOADS[name]
    n = p["n"]
    if p["kind"] == "cd2d_upwind":
        N = n * n
        what = (f"2D upwind convection-diffusion {n}x{n} (N={N}, nnz={5 * N - 4 * n}), Peclet 50")
        if "theta_seed" in p:
            what += f", edge weights theta = 1 + 0.1 N(0,1) seed {p['theta_seed']}"
        return f"{name}: {what}, b~N(0,1) seed {p['b_seed']}"
    if p["kind"] == "cd3d_upwind":
        N = n ** 3
        return (f"{name}: 3D upwind convection-diffusion {n}^3 (N={N}, nnz={7 * N - 6 * n * n}), "
                f"Peclet 50; {p['n_systems']} systems A_i = A + diag(d_i), d_i ~ "
                f"{p['d_scale']:g} U(0,1) seeds {p['d_seed0']}+i, b_i ~ N(0,1) seeds {p['b_seed0']}+i")
    if p["kind"] == "helmholtz2d":
        N = n * n
        return (f"{name}: complex shifted Helmholtz -Laplace - kappa^2 (1 + 0.5i), kappa {p['kappa']:g}, "
                f"{n}x{n} (N={N}, nnz={5 * N - 4 * n}, complex128), b~CN(0,1) seed {p['b_seed']}")
    raise ValueError(p["kind"])


def workload(name: str, n: int | None = None):
    """Return (A, b, params) for a named workload; ``n`` overrides the grid size."""
    p = dict(WORKLOADS[name])
    if n is not None:
        p["n"] = n
    kind = p["kind"]
    if kind == "cd2d_upwind":
        A = cd2d_upwind(p["n"])
        if "theta_seed" in p:
            theta = 1.0 + 0.1 * randn(A.nnz, p["theta_seed"])
            p["theta"] = theta
            p["A0"] = A
            A = edge_weighted(A, theta)
        b = randn(A.n, p.get("b_seed", p.get("b_seed0", 1)))
    elif kind == "cd3d_upwind":
        A = cd3d_upwind(p["n"])
        b = randn(A.n, p["b_seed0"] + 1)
    elif kind == "helmholtz2d":
        A = helmholtz2d(p["n"], p["kappa"])
        b = crandn(A.n, p["b_seed"])
    else:
        raise ValueError(kind)
    return A, b, p


def sequence_system(A0: CSR, p: dict, i: int):
    """System i (1-based) of the shifted sequence A_i = A0 + diag(d_i)."""
    d = p["d_scale"] * np.random.default_rng(p["d_seed0"] + i).uniform(0.0, 1.0, A0.n)
    return shifted_diagonal(A0, d), randn(A0.n, p["b_seed0"] + i)
