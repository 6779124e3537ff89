"""ILU(0) right preconditioning in a multicolour ordering -- test infrastructure only.

Section 6 solves its Stokes systems with ILU preconditioning and leaves the
variant open.  The readings taken here (the GPU library takes the same ones):

* zero fill: the factors L (unit lower) and U (upper) live on the pattern of
  A, and (L U)_ij = A_ij wherever A has an entry (ILU(0));
* right preconditioning: A M^-1 u = b is solved and x = M^-1 u, so the
  residual the method controls is the residual of A x = b itself;
* the unknowns are taken colour by colour: a greedy colouring of the
  symmetrised pattern (vertex i, in increasing index, takes the smallest
  colour that none of its lower-indexed neighbours holds), increasing index
  within a colour.  M = P^T L U P, where L U is the ILU(0) factorisation of
  P A P^T and P the permutation to that order.  (No two neighbours share a
  colour, so the triangular solves advance a whole colour at a time.)

Everything is plain Python / SciPy; it is meant for the test sizes.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .gmres_sdr import SolveResult, sdr_solve


def greedy_colours(A) -> np.ndarray:
    """Colour of each unknown: the smallest colour not held by a neighbour of
    lower index in the symmetrised pattern of A (diagonal ignored)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    S = (P + P.T).tocsr()
    colours = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        used = {int(colours[j]) for j in nb if j < i}
        c = 0
        while c in used:
            c += 1
        colours[i] = c
    return colours


def multicolour_order(colours: np.ndarray) -> np.ndarray:
    """order[p] = the unknown at position p: by colour, then by index."""
    n = colours.shape[0]
    return np.lexsort((np.arange(n), colours))


def ilu0(Ap):
    """ILU(0) of a matrix already in elimination order, row by row: for each
    entry (i, k) left of the diagonal, in increasing k, divide by the pivot
    u_kk and subtract that multiple of row k of U from the entries of row i
    right of k that the pattern holds.  Returns (L, U) as CSR matrices with
    L's unit diagonal stored.  Raises ValueError on a zero pivot."""
    Ap = sp.csr_matrix(Ap)
    n = Ap.shape[0]
    rows = []
    for i in range(n):
        lo, hi = Ap.indptr[i], Ap.indptr[i + 1]
        rows.append({int(c): Ap.data[e] for c, e in zip(Ap.indices[lo:hi], range(lo, hi))})
    urows = []
    for i in range(n):
        row = rows[i]
        for k in sorted(c for c in row if c < i):
            piv = urows[k][k]
            row[k] = row[k] / piv
            lik = row[k]
            for j, ukj in urows[k].items():
                if j > k and j in row:
                    row[j] = row[j] - lik * ukj
        if row.get(i, 0) == 0:
            raise ValueError(f"ILU(0) pivot {i} is zero")
        urows.append({c: v for c, v in row.items() if c >= i})
    dt = Ap.dtype
    Lr, Lc, Lv, Ur, Uc, Uv = [], [], [], [], [], []
    for i in range(n):
        Lr.append(i)
        Lc.append(i)
        Lv.append(1.0)
        for c, v in rows[i].items():
            if c < i:
                Lr.append(i)
                Lc.append(c)
                Lv.append(v)
        for c, v in urows[i].items():
            Ur.append(i)
            Uc.append(c)
            Uv.append(v)
    L = sp.csr_matrix((np.array(Lv, dtype=dt), (Lr, Lc)), shape=(n, n))
    U = sp.csr_matrix((np.array(Uv, dtype=dt), (Ur, Uc)), shape=(n, n))
    return L, U


class ILU0:
    """M = P^T L U P for A in the multicolour order; ``solve`` applies M^-1,
    ``mult`` applies M."""

    def __init__(self, A):
        A = sp.csr_matrix(A)
        self.n = A.shape[0]
        self.colours = greedy_colours(A)
        self.order = multicolour_order(self.colours)
        Ap = A[self.order][:, self.order]
        self.L, self.U = ilu0(Ap)

    def solve(self, v):
        v = np.asarray(v)
        pv = v[self.order]
        y = spla.spsolve_triangular(self.L, pv, lower=True, unit_diagonal=True)
        z = spla.spsolve_triangular(self.U, y, lower=False)
        out = np.empty_like(z)
        out[self.order] = z
        return out

    def mult(self, v):
        v = np.asarray(v)
        pv = v[self.order]
        z = self.L @ (self.U @ pv)
        out = np.empty_like(z)
        out[self.order] = z
        return out


def sdr_solve_right_ilu0(A, b, *, x0=None, **kw) -> SolveResult:
    """GMRES-SDR on the right-preconditioned system (A M^-1) u = b with M the
    multicolour ILU(0) of A; the initial guess is u0 = M x0 and the returned
    ``x`` is M^-1 u.  Keyword arguments as for ``sdr_solve`` (``recycle`` and
    ``new_matrix`` refer to A M^-1)."""
    A = sp.csr_matrix(A)
    M = ILU0(A)
    dt = np.result_type(A.dtype, np.asarray(b).dtype)

    def mv(v):
        return A @ M.solve(np.asarray(v).reshape(-1))

    def mm(V):
        V = np.asarray(V)
        return np.column_stack([mv(V[:, c]) for c in range(V.shape[1])]) if V.shape[1] else \
            np.zeros((A.shape[0], 0), dtype=dt)

    op = spla.LinearOperator(A.shape, matvec=mv, matmat=mm, dtype=dt)
    u0 = None if x0 is None else M.mult(np.asarray(x0, dtype=dt))
    out = sdr_solve(op, b, x0=u0, **kw)
    out.x = M.solve(out.x)
    return out
