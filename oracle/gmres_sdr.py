"""GMRES-SDR oracle in float64 / complex128 -- test infrastructure only.

One restart cycle of GMRES-SDR for A x = r0 is written from Section 3 as
separate parts: the truncated Arnoldi process (Section 3.2), the sketches of
the basis and of A times the basis (Section 3, eq. (3.1)), the sketched
least-squares problem (eq. (3.2), Section 3.3), the residual control
(Section 3.4) and the sketched harmonic-Ritz compression (Section 3.5, eq.
(3.6)); ``sdr_cycle`` composes them, ``sdr_solve`` adds the restart loop and
the sequence variants of Section 3.6.  Every dense small-matrix step uses a
plain NumPy/SciPy routine (lstsq, svd, ordqz); nothing is blocked, fused or
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
  that column is taken as dependent and left out of the least squares (its
  coefficient is zero, the sketched residual is the previous step's), the
  check is forced and the cycle ends.
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
from .srdct import SRDCT


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
    est: float = float("nan")  # Givens estimate (Givens control only)
    eps: float = float("nan")  # its eps before the check


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
    eps: float = float("nan")  # fitted eps of the Givens control
    refits: list = field(default_factory=list)  # its eps refits


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


def _window(j: int, t: int) -> range:
    """1-based indices of the basis vectors that the j-th new direction is
    orthogonalised against: the t most recent ones, v_{j-t+1} .. v_j
    (Section 3.2; fewer at the start of a cycle)."""
    return range(max(j - t + 1, 1), j + 1)


def arnoldi_extend(A, V, H, j: int, t: int, breakdown_rtol: float, bump) -> bool:
    """Truncated Arnoldi (Section 3.2): append v_{j+1} to V.

    w = A v_j loses its components along the window vectors one after the
    other (modified Gram-Schmidt in increasing index, coefficients H(i, j) =
    v_i^* w, conjugate-linear in v_i); H(j+1, j) = ||w|| and v_{j+1} =
    w / H(j+1, j), so that A V_j = V_{j+1} H_j with H banded.  Returns True on
    breakdown, H(j+1, j) <= breakdown_rtol * ||A v_j||, in which case no
    v_{j+1} is formed and H(j+1, j) = 0.
    """
    w = A @ V[:, j - 1]
    bump("matvecs")
    norm_Av = _norm(w)
    for i in _window(j, t):
        hij = np.vdot(V[:, i - 1], w)
        bump("inner_products")
        H[i - 1, j - 1] = hij
        w = w - V[:, i - 1] * hij
    hn = _norm(w)
    bump("inner_products")
    if not (hn > breakdown_rtol * norm_Av):
        H[j, j - 1] = 0.0
        return True
    H[j, j - 1] = hn
    V[:, j] = w / hn
    return False


def sketch_extend(S, V, H, SV, SAV, j: int, breakdown: bool, bump) -> None:
    """Sketches of step j (Section 3): the new basis vector is sketched once,
    SV(:, j+1) = S v_{j+1}, and S A v_j needs no sketch of its own, since the
    Arnoldi relation gives A v_j = V_{j+1} H(:, j), hence
    S A v_j = SV(:, 1:j+1) H(1:j+1, j) (only the band is nonzero)."""
    nc = j if breakdown else j + 1
    if not breakdown:
        SV[:, j] = S @ V[:, j]
        bump("sketches")
    SAV[:, j - 1] = SV[:, :nc] @ H[:nc, j - 1]


def sketched_least_squares(SAW, Sr):
    """Sketched minimal residual (eq. (3.2)): the minimum-norm y minimising
    ||S r0 - SAW y||, and that minimum, the sketched residual norm."""
    y, *_ = np.linalg.lstsq(SAW, Sr, rcond=None)
    return y, _norm(Sr - SAW @ y)


def newest_column_dependent(SAW, rank_rtol: float) -> bool:
    """True if the last column of SAW lies within rank_rtol (relative) of the
    span of the others: the sketched basis of the search space lost rank."""
    a = SAW[:, -1]
    na = _norm(a)
    if SAW.shape[1] == 1 or na == 0:
        return not (na > 0)
    c, *_ = np.linalg.lstsq(SAW[:, :-1], a, rcond=None)
    return not (_norm(a - SAW[:, :-1] @ c) / na > rank_rtol)


class SafetyControl:
    """Residual control of Section 3.4: the true residual is evaluated once
    the sketched one falls below tol / safety; a failed evaluation raises
    safety to the observed ratio ||r|| / ||S r||."""

    def __init__(self, safety: float):
        self.safety = safety

    def due(self, sres: float, tol_abs: float) -> bool:
        return sres < tol_abs / self.safety

    def failed(self, sres: float, res: float) -> None:
        if sres > 0:
            self.safety = res / sres


def givens_sine(SAU, SV, H, j: int) -> float:
    """|s_j|, the sine of the j-th Givens rotation of the QR factorisation of
    the augmented Hessenberg matrix of Section 5.

    With [SAU, SV(:, 1:j+1)] = W R (economy QR), S A [U, V_j] = W G_j where
    G_j = R blkdiag(I, H_j): its first k columns are already triangular and
    the rest, R22 H_j, is upper Hessenberg, so one Givens rotation per
    Arnoldi step triangularises it.  Built here from scratch at every step.
    """
    kh = SAU.shape[1]
    _, R = np.linalg.qr(np.concatenate([SAU, SV[:, : j + 1]], axis=1))
    B = np.zeros((kh + j + 1, kh + j), dtype=R.dtype)
    B[:kh, :kh] = np.eye(kh)
    B[kh:, kh:] = H[: j + 1, :j]
    G = R @ B
    s_last = 0.0
    for i in range(j):  # rotation i acts on rows kh+i, kh+i+1
        c0 = kh + i
        a, b = G[c0, c0], G[c0 + 1, c0]
        r = np.hypot(abs(a), abs(b))
        if r == 0.0:
            s_last = 0.0
            continue
        cs = abs(a) / r
        sn = (a / abs(a) if a != 0 else 1.0) * np.conj(b) / r
        rows = G[c0 : c0 + 2, c0:].copy()
        G[c0, c0:] = cs * rows[0] + sn * rows[1]
        G[c0 + 1, c0:] = -np.conj(sn) * rows[0] + cs * rows[1]
        s_last = abs(b) / r
    return float(s_last)


def givens_factor(sine: float, eps: float) -> float:
    """Growth factor of the true-residual estimate over one step (Section 4.5,
    the corollary to the Givens-sine theorem): ||r_j|| <= sqrt((s_j^2 +
    2 eps (1 + c_j)) / (1 - eps^2)) ||r_{j-1}||, with c_j = sqrt(1 - s_j^2),
    evaluated at the sketched sine (the computable one)."""
    c = np.sqrt(max(0.0, 1.0 - sine * sine))
    return float(np.sqrt((sine * sine + 2.0 * eps * (1.0 + c)) / (1.0 - eps * eps)))


class GivensControl:
    """Residual control by the Givens-rotation estimate (Sections 4.5 and 5).

    The estimate starts each cycle from ||r0|| (no recycled block) or from
    the U-only sketched residual divided by sqrt(1 - eps) (the bound eq. (3.5)
    gives for the sketched minimiser), and is multiplied by givens_factor at
    every step.  The true residual is evaluated once the estimate falls below
    the tolerance.  When a true residual exceeds its estimate, eps is raised to
    the smallest value for which the estimate, restarted from the last anchor
    (the cycle start or the previous true residual), reaches it; the estimate
    then restarts from the true residual.  eps persists across cycles.
    """

    def __init__(self, eps: float):
        self.eps = float(eps)
        self.est = np.inf
        self.sines = []        # sines since the anchor
        self.anchor = None     # (value, depends_on_eps) of the anchor
        self.safety = np.nan   # (recorded with the checks)
        self.refits = []       # (res, eps before, eps after, estimates at the bracket ends)

    def start(self, beta: float, sres0: float, khat: int) -> None:
        if khat == 0:
            self.anchor = (beta, False)
        else:
            self.anchor = (sres0, True)
        self.sines = []
        self.est = self._estimate(self.eps)

    def _estimate(self, eps: float) -> float:
        v, scaled = self.anchor
        e = v / np.sqrt(1.0 - eps) if scaled else v
        for sn in self.sines:
            e *= givens_factor(sn, eps)
        return e

    def step(self, sine: float) -> None:
        self.sines.append(sine)
        self.est *= givens_factor(sine, self.eps)

    def due(self, sres: float, tol_abs: float) -> bool:
        return self.est < tol_abs

    def failed(self, sres: float, res: float) -> None:
        self.checked(res)

    def checked(self, res: float) -> None:
        """A true residual res at this step: refit eps if the estimate fell
        short of it, then restart the estimate from res."""
        if res > self._estimate(self.eps):
            lo, hi = self.eps, 1.0
            for _ in range(200):  # bisection: the estimate grows with eps
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                if self._estimate(mid) >= res:
                    hi = mid
                else:
                    lo = mid
            self.refits.append((res, self.eps, hi, self._estimate(hi), self._estimate(lo)))
            self.eps = hi
        self.anchor = (res, False)
        self.sines = []
        self.est = res


def sdr_cycle(A, S, r0, rec: Recycle, tol_abs: float, m: int, t: int, k: int,
              safety: float, *, breakdown_rtol=1e-14, rank_rtol=1e-12,
              counters=None, keep=None, control=None):
    """One restart cycle of GMRES-SDR for the correction equation A x = r0.

    The search space is [U, V_j]: the recycle block and the truncated Arnoldi
    basis of K_j(A, r0), grown one vector at a time (arnoldi_extend).  After
    each step the sketched least-squares problem over it is solved
    (sketched_least_squares); the residual control of Section 3.4 decides
    when the true residual is evaluated, and the cycle stops on convergence,
    at j = m, at an Arnoldi breakdown or when the sketched basis loses rank.
    Finally the recycle triple is compressed by harmonic_ritz_update.

    ``control`` is the residual control (SafetyControl(safety) when None, or
    a GivensControl carried across cycles).  Returns (xt, rt, res,
    new_recycle, record, safety).  If ``keep`` is a dict it receives the
    cycle's V, H, SV, SAV, y and G for inspection.
    """
    N = r0.shape[0]
    s = S.shape[0]
    dt = np.result_type(r0.dtype, rec.U.dtype, A.dtype)
    real = not np.iscomplexobj(np.zeros(0, dtype=dt))
    cnt = counters if counters is not None else {}

    def bump(key, v=1):
        cnt[key] = cnt.get(key, 0) + v

    U, SU, SAU = rec.U, rec.SU, rec.SAU
    # the cycle starts from v_1 = r0 / ||r0|| and its sketch S r0 / ||r0||
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
    if control is None:
        control = SafetyControl(safety)
    givens = isinstance(control, GivensControl)
    if givens:
        # the sketched residual over span(U) alone, where the estimate starts
        sres0 = sketched_least_squares(SAU, Sr)[1] if U.shape[1] > 0 else _norm(Sr)
        control.start(beta, sres0, U.shape[1])

    rec_out = CycleRecord(0, np.inf, np.inf, False, False, False, 0, 0)
    xt = None
    rt = None
    res = np.inf
    j_stop = m
    for j in range(1, m + 1):
        breakdown = arnoldi_extend(A, V, H, j, t, breakdown_rtol, bump)
        sketch_extend(S, V, H, SV, SAV, j, breakdown, bump)
        bump("iters")
        SAW = np.concatenate([SAU, SAV[:, :j]], axis=1)
        rank_loss = newest_column_dependent(SAW, rank_rtol)
        if rank_loss:
            # a column declared dependent adds no direction: the least squares
            # runs over the others and its coefficient is zero
            y, sres = sketched_least_squares(SAW[:, :-1], Sr)
            y = np.concatenate([y, np.zeros(1, dtype=y.dtype)])
        else:
            y, sres = sketched_least_squares(SAW, Sr)
        rec_out.sres_hist.append(sres)
        if givens:
            control.step(givens_sine(SAU, SV, H, j))
        if not (control.due(sres, tol_abs) or j == m or breakdown or rank_loss):
            continue
        # true residual of the iterate from the search space
        xt = np.concatenate([U, V[:, :j]], axis=1) @ y
        rt = r0 - A @ xt
        bump("matvecs")
        res = _norm(rt)
        bump("inner_products")
        bump("res_checks")
        rec_out.checks.append(Check(j, sres, res, control.safety,
                                    control.est if givens else float("nan"),
                                    control.eps if givens else float("nan")))
        j_stop = j
        if res < tol_abs:
            rec_out.converged = True
            break
        if breakdown or rank_loss:
            break
        control.failed(sres, res)
    rec_out.j_stop = j_stop
    rec_out.sres = rec_out.sres_hist[-1]
    rec_out.res = res
    rec_out.breakdown = bool(breakdown)
    rec_out.rank_loss = bool(rank_loss)

    # compression of the search space into the next recycle triple, also
    # after convergence (a sequence reuses it)
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
    return xt, rt, res, new, rec_out, control.safety


def sdr_solve(A, b, *, x0=None, m: int, k: int, t: int, s: int, zeta: int = 8,
              seed: int = 42, tol: float = 1e-8, safety0: float = 1.4,
              max_cycles: int = 10000, recycle: Recycle | None = None,
              new_matrix: bool = False, variant: str = "exact",
              persist_safety: bool = False, S=None,
              breakdown_rtol: float = 1e-14, rank_rtol: float = 1e-12,
              keep_cycles: list | None = None, resid_control: str = "safety",
              givens_eps0: float = 0.0, sketch: str = "sparse_sign") -> SolveResult:
    """Restarted GMRES-SDR for A x = b (relative tolerance ``tol``).

    ``recycle`` carries U, SU, SAU from a previous solve; ``new_matrix`` says
    that A differs from the matrix SAU was formed with (Section 3.6).
    ``resid_control`` "safety" (Section 3.4) or "givens" (the Givens-rotation
    estimate of Sections 4.5 and 5 with eps fitted to the true residuals,
    starting from ``givens_eps0``; the fitted eps is returned as ``eps``).
    ``sketch`` "sparse_sign" (zeta nonzeros per column) or "srdct" (the
    subsampled randomised DCT of Section 6); an explicit ``S`` overrides it.
    """
    if A.dtype.kind == "c" or np.iscomplexobj(b):
        dt = np.complex128
    else:
        dt = np.float64
    N = b.shape[0]
    if S is None:
        if sketch == "srdct":
            S = SRDCT(N, s, seed)
        elif sketch == "sparse_sign":
            S = sketch_operator(N, s, zeta, seed)
        else:
            raise ValueError("sketch is 'sparse_sign' or 'srdct'")
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
    if resid_control not in ("safety", "givens"):
        raise ValueError("resid_control is 'safety' or 'givens'")
    gctl = GivensControl(givens_eps0) if resid_control == "givens" else None
    converged = rn <= tol_abs
    cyc = 0
    while not converged and cyc < max_cycles:
        if not persist_safety:
            safety = safety0
        keep = {} if keep_cycles is not None else None
        xt, rt, res, recycle, rec, safety = sdr_cycle(
            A, S, r, recycle, tol_abs, m, t, k, safety,
            breakdown_rtol=breakdown_rtol, rank_rtol=rank_rtol, counters=cnt,
            keep=keep, control=gctl)
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
    out.eps = gctl.eps if gctl is not None else float("nan")
    out.refits = gctl.refits if gctl is not None else []
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
