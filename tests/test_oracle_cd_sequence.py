"""The oracle's stored run of the paper's last experiment (Section 6.3,
Table 4; tests/golden/cd2d_central_seq.json, written from the oracle by
tests/golden/make_cd2d_central_seq.py) shows the paper's finding: the exact
variant converges on all three systems, the inexact one on the first two
only, and on the third its true residual grows while every cycle still ends
with a sketched residual below the residual it started from."""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "cd2d_central_seq.json")) as f:
    GOLD = json.load(f)
P = GOLD["params"]


def _sketched_below_start(trace, nb):
    start = nb
    for c in trace:
        if not c["sres"] < start:
            return False
        start = c["res"]
    return True


def test_golden_pins_the_papers_finding():
    nb = float(P["n"])  # ||ones|| on n^2 entries
    for g in GOLD["runs"]["exact"]:
        assert g["converged"] and g["relres"] <= P["tol"]
    inexact = GOLD["runs"]["inexact"]
    assert inexact[0]["converged"] and inexact[1]["converged"]
    third = inexact[2]
    assert not third["converged"]
    res = [c["res"] for c in third["trace"]]
    assert res[-1] > 100.0 * res[0] and res[-1] > nb
    assert _sketched_below_start(third["trace"], nb)


