"""GMRES-SDR oracle in float64 / complex128 -- test infrastructure only.

Follows the paper's Algorithm 1 (one cycle of GMRES-SDR for A x = r0) step by
step, in the paper's order and notation, plus the restart loop and the
sequence variants of Section 3.6.  Every dense small-matrix step uses a plain
NumPy/SciPy routine (lstsq, svd, ordqz); nothing is blocked, fused or
reordered.  Where the paper is silent the following readings are taken (the
GPU library takes the same ones):

* m counts Arnoldi steps per cycle; the search space is [U, V(:, 1:j)].
* tol is relative: the absolute target is tol * ||b||.
* Truncated Arnoldi orthogonalises against the t most recent basis vectors
  v_max(j-t+1,1) .. v_j by modified Gram-Schmidt in increasing order; inner
  products are conjugate-linear in the first argument (Algorithm 1, 3.1).
* The sketched basis is initialised as [S r0/||r0||, 0_{s x m}].
* ``safety`` restarts at ``safety0`` (1.4) in every cycle unless
  ``persist_safety``; it is raised to res/sres after a failed true-residual
  check (Section 3.4).
* Arnoldi breakdown, H(j+1,j) <= breakdown_rtol * ||A v_j||: no v_{j+1} is
  formed, the true-residual check is forced at this j and the cycle ends.
* Rank loss of the sketched least-squares matrix, i.e. the new column of
  SAW lies within rank_rtol (relative) of the span of the previous columns:
  the minimum-norm solution is kept, the check is forced and the cycle ends.
* The recycle space is refreshed after every cycle, converged or not
  (Algorithm 1 reaches the update after ``break``).  Its input "SW" is the
  sketched search basis [SU, SV(:, 1:j)], and V(:, 1:m) there means the j
  columns built in the cycle.
* Truncated SVD: ell = #{sigma_i > sigma_1 * max(s, khat+j) * 2^-52}.
* Ordered QZ of the pencil (M_ell, Sigma_ell): the k eigenvalues mu = alpha /
  beta of largest modulus (ties by QZ position) are moved to the top; for real
  data a conjugate pair is never split, so k_eff may be k + 1.
* Sequences (Section 3.6): with the same A the recycle triple is passed on;
  after a change of A the exact variant recomputes SAU = S (A U) (k extra
  products and sketches), the inexact variant keeps the stale SAU.
* Right preconditioning (Section 6 solves preconditioned systems; the
  Jacobi case): A x = b is solved as (A D^-1) u = b with D = diag(A) and
  x = D^-1 u, so the residual b - (A D^-1) u is that of A x = b and the
  recycle triple belongs to A D^-1.  ``sdr_solve_right_jacobi``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .sketch import sketch_operator


@dataclass
class Recycle:
    """Recycle triple U (N x khat), SU = S U, SAU = S A U (s x khat)."""

    U: np.ndarray
    SU: np.ndarray
    SAU: np.ndarray

    @property
    def k(self) -> int:
        return self.U.shape[1]


@dataclass
class Check:
    j: int
    sres: float
    res: float
    safety: float


@dataclass
class CycleRecord:
    j_stop: int
    sres: float
    res: float
    converged: bool
    breakdown: bool
    rank_loss: bool
    ell: int
    k_eff: int
    checks: list = field(default_factory=list)
    sres_hist: list = field(default_factory=list)


@dataclass
class SolveResult:
    x: np.ndarray
    converged: bool
    relres: float
    cycles: int = 0
    iters: int = 0
    matvecs: int = 0
    inner_products: int = 0
    sketches: int = 0
    res_checks: int = 0
    trace: list = field(default_factory=list)
    recycle: Recycle | None = None


def _norm(v) -> float:
    return float(np.linalg.norm(v))


def harmonic_ritz_update(W, SB, SAW, k: int, real: bool, s: int):
    """Sketched harmonic-Ritz compression (Section 3.5, eq. (3.6)).

    W = [U, V(:,1:j)] (N x ell0), SB = its sketch, SAW = S A W.
    Returns (G, ell, k_eff) with G = Vhat_ell Z(:, 1:k_eff), so that the new
    recycle triple is W G, SB G, SAW G.
    """
    ell0 = SAW.shape[1]
    P, sig, Wh = np.linalg.svd(SAW, full_matrices=False)
    if ell0 == 0 or sig[0] == 0.0:
        return np.zeros((ell0, 0), dtype=SAW.dtype), 0, 0
    ell = int(np.count_nonzero(sig > sig[0] * max(s, ell0) * 2.0 ** -52))
    Uh = P[:, :ell]
    Vh = Wh.conj().T[:, :ell]
    Sig = np.diag(sig[:ell]).astype(SAW.dtype)
    M = Uh.conj().T @ SB @ Vh
    kk = min(k, ell)
    info = {}

    def select(alpha, beta):
        mod = np.abs(alpha) / np.abs(beta)
        order = np.argsort(-mod, kind="stable")
        sel = np.zeros(alpha.shape[0], dtype=bool)
        sel[order[:kk]] = True
        if real:  # never split a complex-conjugate pair
            ai = np.imag(alpha)
            for i in np.nonzero(sel)[0]:
                if ai[i] > 0:
                    sel[i + 1] = True
                elif ai[i] < 0:
                    sel[i - 1] = True
        info["k_eff"] = int(sel.sum())
        return sel

    out = "real" if real else "complex"
    if real:
        M = M.real
        Sig = Sig.real
    _, _, _, _, _, Z = sla.ordqz(M, Sig, sort=select, output=out)
    k_eff = info["k_eff"]
    G = Vh @ Z[:, :k_eff]
    return G, ell, k_eff


def sdr_cycle(A, S, r0, rec: Recycle, tol_abs: float, m: int, t: int, k: int,
              safety: float, *, breakdown_rtol=1e-14, rank_rtol=1e-12,
              counters=None, keep=None):
    """One cycle of Algorithm 1 for A x = r0.

    Returns (xt, rt, res, new_recycle, record, safety).  If ``keep`` is a
    dict it receives the cycle's V, H, SV, SAV, y and G for inspection.
    """
    N = r0.shape[0]
    s = S.shape[0]
    dt = np.result_type(r0.dtype, rec.U.dtype, A.dtype)
    real = not np.iscomplexobj(np.zeros(0, dtype=dt))
    cnt = counters if counters is not None else {}

    def bump(key, v=1):
        cnt[key] = cnt.get(key, 0) + v

    U, SU, SAU = rec.U, rec.SU, rec.SAU
    khat = U.shape[1]
    # sketch of the initial residual; basis and sketched basis (Alg. 1)
    Sr = S @ r0
    bump("sketches")
    beta = _norm(r0)
    bump("inner_products")
    V = np.zeros((N, m + 1), dtype=dt)
    V[:, 0] = r0 / beta
    H = np.zeros((m + 1, m), dtype=dt)
    SV = np.zeros((s, m + 1), dtype=dt)
    SV[:, 0] = Sr / beta
    SAV = np.zeros((s, m), dtype=dt)

    rec_out = CycleRecord(0, np.inf, np.inf, False, False, False, 0, 0)
    xt = None
    rt = None
    res = np.inf
    j_stop = m
    for j in range(1, m + 1):
        # --- truncated Arnoldi (MGS against the t most recent vectors) ---
        w = A @ V[:, j - 1]
        bump("matvecs")
        norm_Av = _norm(w)
        for i in range(max(j - t + 1, 1), j + 1):
            H[i - 1, j - 1] = np.vdot(V[:, i - 1], w)
            bump("inner_products")
            w = w - V[:, i - 1] * H[i - 1, j - 1]
        hn = _norm(w)
        bump("inner_products")
        breakdown = not (hn > breakdown_rtol * norm_Av)
        if not breakdown:
            H[j, j - 1] = hn
            V[:, j] = w / hn
            SV[:, j] = S @ V[:, j]  # one sketch per iteration
            bump("sketches")
            # sketch of A v_j from the Arnoldi relation, no extra sketch
            SAV[:, j - 1] = SV[:, : j + 1] @ H[: j + 1, j - 1]
        else:
            H[j, j - 1] = 0.0
            SAV[:, j - 1] = SV[:, :j] @ H[:j, j - 1]
        bump("iters")
        SAW = np.concatenate([SAU, SAV[:, :j]], axis=1)
        # --- sketched least squares (minimum-norm solution) ---
        y, *_ = np.linalg.lstsq(SAW, Sr, rcond=None)
        sres = _norm(Sr - SAW @ y)
        rec_out.sres_hist.append(sres)
        # rank test of the appended column against the previous ones
        a = SAW[:, -1]
        Pm = SAW[:, :-1]
        na = _norm(a)
        if Pm.shape[1] > 0 and na > 0:
            c, *_ = np.linalg.lstsq(Pm, a, rcond=None)
            dist = _norm(a - Pm @ c) / na
        else:
            dist = 1.0 if na > 0 else 0.0
        rank_loss = not (dist > rank_rtol)
        # --- residual control (Section 3.4) ---
        if sres < tol_abs / safety or j == m or breakdown or rank_loss:
            Wb = np.concatenate([U, V[:, :j]], axis=1)
            xt = Wb @ y
            rt = r0 - A @ xt
            bump("matvecs")
            res = _norm(rt)
            bump("inner_products")
            bump("res_checks")
            rec_out.checks.append(Check(j, sres, res, safety))
            if res < tol_abs:
                rec_out.converged = True
                j_stop = j
                break
            if breakdown or rank_loss:
                j_stop = j
                break
            if sres > 0:
                safety = res / sres
            if j == m:
                j_stop = j
                break
    rec_out.j_stop = j_stop
    rec_out.sres = rec_out.sres_hist[-1]
    rec_out.res = res
    rec_out.breakdown = bool(breakdown)
    rec_out.rank_loss = bool(rank_loss)

    # --- harmonic-Ritz update of the recycle space (always) ---
    j = j_stop
    SAW = np.concatenate([SAU, SAV[:, :j]], axis=1)
    SB = np.concatenate([SU, SV[:, :j]], axis=1)
    Wb = np.concatenate([U, V[:, :j]], axis=1)
    G, ell, k_eff = harmonic_ritz_update(Wb, SB, SAW, k, real, s)
    rec_out.ell, rec_out.k_eff = ell, k_eff
    new = Recycle(Wb @ G, SB @ G, SAW @ G)
    if keep is not None:
        keep.update(V=V[:, : j + 1], H=H[: j + 1, :j], SV=SV[:, : j + 1],
                    SAV=SAV[:, :j], y=y, G=G, Sr=Sr, j=j, xt=xt,
                    U_in=U, SU_in=SU, SAU_in=SAU)
    return xt, rt, res, new, rec_out, safety


def sdr_solve(A, b, *, x0=None, m: int, k: int, t: int, s: int, zeta: int = 8,
              seed: int = 42, tol: float = 1e-8, safety0: float = 1.4,
              max_cycles: int = 10000, recycle: Recycle | None = None,
              new_matrix: bool = False, variant: str = "exact",
              persist_safety: bool = False, S=None,
              breakdown_rtol: float = 1e-14, rank_rtol: float = 1e-12,
              keep_cycles: list | None = None) -> SolveResult:
    """Restarted GMRES-SDR for A x = b (relative tolerance ``tol``).

    ``recycle`` carries U, SU, SAU from a previous solve; ``new_matrix`` says
    that A differs from the matrix SAU was formed with (Section 3.6).
    """
    if A.dtype.kind == "c" or np.iscomplexobj(b):
        dt = np.complex128
    else:
        dt = np.float64
    N = b.shape[0]
    if S is None:
        S = sketch_operator(N, s, zeta, seed)
    b = np.asarray(b, dtype=dt)
    x = np.zeros(N, dtype=dt) if x0 is None else np.array(x0, dtype=dt)
    cnt: dict = {}
    out = SolveResult(x=x, converged=False, relres=np.inf)
    if recycle is None:
        recycle = Recycle(np.zeros((N, 0), dt), np.zeros((s, 0), dt), np.zeros((s, 0), dt))
    else:
        recycle = Recycle(recycle.U.astype(dt), recycle.SU.astype(dt), recycle.SAU.astype(dt))
        if new_matrix and variant == "exact" and recycle.k > 0:
            AU = A @ recycle.U
            cnt["matvecs"] = cnt.get("matvecs", 0) + recycle.k
            recycle.SAU = S @ AU
            cnt["sketches"] = cnt.get("sketches", 0) + recycle.k
    nb = _norm(b)
    tol_abs = tol * nb
    r = b - A @ x
    cnt["matvecs"] = cnt.get("matvecs", 0) + 1
    rn = _norm(r)
    cnt["inner_products"] = cnt.get("inner_products", 0) + 1
    if nb == 0.0:
        out.x, out.converged, out.relres = np.zeros(N, dt), True, 0.0
        out.recycle = recycle
        return out
    safety = safety0
    converged = rn <= tol_abs
    cyc = 0
    while not converged and cyc < max_cycles:
        if not persist_safety:
            safety = safety0
        keep = {} if keep_cycles is not None else None
        xt, rt, res, recycle, rec, safety = sdr_cycle(
            A, S, r, recycle, tol_abs, m, t, k, safety,
            breakdown_rtol=breakdown_rtol, rank_rtol=rank_rtol, counters=cnt,
            keep=keep)
        if keep_cycles is not None:
            keep.update(r0=r, U=recycle.U)
            keep_cycles.append(keep)
        cyc += 1
        x = x + xt
        r = rt
        rn = res
        out.trace.append(rec)
        converged = rec.converged
        if (rec.breakdown or rec.rank_loss) and not converged and rec.j_stop == 1:
            break  # no progress possible
    out.x = x
    out.converged = bool(converged)
    out.relres = rn / nb
    out.cycles = cyc
    out.iters = cnt.get("iters", 0)
    out.matvecs = cnt.get("matvecs", 0)
    out.inner_products = cnt.get("inner_products", 0)
    out.sketches = cnt.get("sketches", 0)
    out.res_checks = cnt.get("res_checks", 0)
    out.recycle = recycle
    return out


def sdr_solve_right_jacobi(A, b, *, x0=None, **kw) -> SolveResult:
    """GMRES-SDR on the right Jacobi preconditioned system (A D^-1) u = b.

    D = diag(A) (every diagonal entry must be nonzero); the initial guess is
    u0 = D x0 and the returned ``x`` is D^-1 u.  Keyword arguments as for
    ``sdr_solve``, with ``recycle`` / ``new_matrix`` referring to A D^-1.
    """
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    d = A.diagonal()
    if np.any(d == 0):
        raise ValueError("Jacobi preconditioning needs a nonzero diagonal")
    dinv = 1.0 / d
    # A D^-1 on A's own pattern and entry order: stored entry (i, j) times 1/d_j
    Ahat = A.copy()
    Ahat.data = A.data * dinv[A.indices]
    u0 = None if x0 is None else d * np.asarray(x0)
    out = sdr_solve(Ahat, b, x0=u0, **kw)
    out.x = out.x / d
    return out
