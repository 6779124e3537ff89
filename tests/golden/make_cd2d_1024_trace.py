"""Writes cd2d_1024_trace.json: the oracle's complete solve of the 1024 x 1024
upwind convection-diffusion system (N = 1,048,576, Peclet 50, b ~ N(0,1) with
seed 1; m = 100, k = 20, t = 2, s = 240, zeta = 8, sketch seed 42, relative
tolerance 1e-8, from x0 = 0).  Stored per cycle: the decisions (stop index,
number of true-residual checks, numerical rank ell, recycle dimension) and the
sketched and true residual norms at the stop; for the solution: its norm, its
entries at 2048 seeded indices and its inner product with a seeded N(0,1)
vector g.  Calls the oracle only (about 8 minutes on 8 cores):

    python tests/golden/make_cd2d_1024_trace.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sdr_solve  # noqa: E402
from workloads import workload, randn  # noqa: E402

SAMPLE_SEED = 77  # indices of the stored entries of x
G_SEED = 78       # the vector g of the stored x . g
N_SAMPLE = 2048


def sample_indices(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, N_SAMPLE, replace=False))


def run():
    A, b, p = workload("cd2d_1024")
    t0 = time.time()
    r = sdr_solve(A.to_scipy(), b, m=p["m"], k=p["k"], t=p["t"], s=p["s"], zeta=p["zeta"],
                  seed=p["s_seed"], tol=p["tol"])
    sec = time.time() - t0
    idx = sample_indices(A.n)
    g = randn(A.n, G_SEED)
    return dict(
        workload="cd2d_1024", params={k: p[k] for k in ("n", "m", "k", "t", "s", "zeta", "tol",
                                                         "b_seed", "s_seed")},
        oracle_seconds=sec, converged=bool(r.converged), relres=float(r.relres), cycles=r.cycles,
        iters=r.iters, matvecs=r.matvecs, inner_products=r.inner_products,
        res_checks=r.res_checks,
        trace=[dict(j_stop=c.j_stop, n_checks=len(c.checks), ell=c.ell, k_eff=c.k_eff,
                    sres=float(c.sres), res=float(c.res)) for c in r.trace],
        x_norm=float(np.linalg.norm(r.x)), x_dot_g=float(r.x @ g),
        sample_seed=SAMPLE_SEED, g_seed=G_SEED, x_sample=[float(v) for v in r.x[idx]])


if __name__ == "__main__":
    data = run()
    print(data["cycles"], data["iters"], data["relres"], "%.0f s" % data["oracle_seconds"])
    with open(os.path.join(HERE, "cd2d_1024_trace.json"), "w") as f:
        json.dump(data, f, indent=1)
