"""Writes cd2d_central_seq.json: the oracle's run of the convection-diffusion
sequence of the paper's last experiment (Section 6.3, Table 4): central
differences on an n = 500 grid, convection strengths 0, 5 and 20, b = ones,
m = 80, k = 20, a target relative residual of 1e-2, with the exact and the
inexact treatment of S A U between systems (Section 3.6).  Truncation t = 2
and a sparse-sign sketch of s = 8 m rows stand in for the paper's settings.
Calls the oracle only:

    python tests/golden/make_cd2d_central_seq.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sdr_solve  # noqa: E402
from oracle.sketch import sketch_operator  # noqa: E402
from workloads.problems import cd2d_central  # noqa: E402

PARAMS = dict(n=500, alphas=[0.0, 5.0, 20.0], m=80, k=20, t=2, s=640, zeta=8, seed=42, tol=1e-2,
              max_cycles=12)


def run():
    p = PARAMS
    N = p["n"] ** 2
    S = sketch_operator(N, p["s"], p["zeta"], p["seed"])
    b = np.ones(N)
    out = dict(params=p, runs={})
    for variant in ("exact", "inexact"):
        rec, systems = None, []
        for alpha in p["alphas"]:
            A = cd2d_central(p["n"], alpha).to_scipy()
            r = sdr_solve(A, b, m=p["m"], k=p["k"], t=p["t"], s=p["s"], S=S, tol=p["tol"],
                          max_cycles=p["max_cycles"], recycle=rec, new_matrix=rec is not None,
                          variant=variant)
            systems.append(dict(
                alpha=alpha, converged=bool(r.converged), relres=float(r.relres), cycles=r.cycles,
                matvecs=r.matvecs, inner_products=r.inner_products,
                trace=[dict(j_stop=c.j_stop, n_checks=len(c.checks), k_eff=c.k_eff, ell=c.ell,
                            sres=float(c.sres), res=float(c.res)) for c in r.trace]))
            print(variant, alpha, systems[-1]["converged"], "%.3e" % r.relres, r.cycles, flush=True)
            rec = r.recycle
        out["runs"][variant] = systems
    return out


if __name__ == "__main__":
    data = run()
    with open(os.path.join(HERE, "cd2d_central_seq.json"), "w") as f:
        json.dump(data, f, indent=1)
