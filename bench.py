"""GMRES-SDR benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cd2d_1024]

A step is one complete solve to a 1e-8 relative residual, from x0 = 0 and an
empty recycle space, of the 2D upwind convection-diffusion operator on a
1024 x 1024 grid (N = 1,048,576, nnz = 5,238,784, Peclet 50, b ~ N(0,1) seed 1)
with m = 100, k = 20, t = 2, s = 240 (zeta = 8) in FP64.  Inputs are resident
in HBM before the timed region.  Prints one JSON line:

* value: median time to 1e-8 (s) over the K timed solves;
* roofline: the SpMV + window-product + sketch kernel (the largest per-step kernel),
  algorithmic bytes per launch / its mean duration from HIP events recorded
  by the dispatches themselves on the library's stream inside the timed
  region, on every 64th Arnoldi step (--timing-every; each timed step costs
  its event records, so sampling is kept sparse);
* roofline.traffic: HBM bytes per launch of that kernel from rocprofv3
  FETCH_SIZE and WRITE_SIZE counters, scaled by what the same counters read
  for a device copy of known size, taken from the committed summary
  profiles/<kernel>_<workload>_hbm_traffic.md; null when the kernel sources
  differ from the ones the counters were taken on (a digest of the sources is
  stored with the figures);
* cpu_baseline: the FP64 oracle on the host cores, timed on the first
  cycle (no recycled block) and the second (k recycled vectors, the steady
  state of every later cycle) of the same solve, extrapolated to the GPU
  solve's steps (the first cycle's cost once, the second's per step after);
* sequence: the 20 slowly changing 3D systems (128^3, N = 2,097,152) solved
  in turn with the recycle space carried (exact variant), in FP64 and with
  the FP32 basis: solves/s, steps per system, the FP64 residual recomputed on
  the host, the first cycle's x against the oracle's, and the step kernel's
  bandwidth (its per-step working set exceeds the 256 MB last-level cache);
* helmholtz: the complex shifted Helmholtz system (1024^2) to 1e-8 in
  complex128 and with the complex64 basis: time, steps, host eigen-step time,
  the host residual and the first cycle's x against the oracle's;
* srdct: the 1024^2 solve with the subsampled randomised DCT sketch of
  Section 6: time, steps, host residual, first-cycle x against the oracle's,
  and the DCT kernel's duration against the FP64 vector issue rate.

    python bench.py --summarize-pmc FETCH.csv WRITE.csv --copy-calib-mb 256

writes that summary (markdown) from the counter CSVs of two rocprofv3 runs of
this script with --copy-calib-mb (one --pmc FETCH_SIZE, one --pmc WRITE_SIZE).

    python bench.py --summarize-kstats STATS.csv TRACE.csv BENCH.json

writes the kernel-statistics summary of a rocprofv3 --kernel-trace --stats run
of this script, next to the kernel duration the bench's own events measured
(BENCH.json: this script's output line from the same machine).
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 rel. residual (s), solves/s on sequences; HBM GB/s of SpMV+sketch"
HBM_PEAK_GBS = 8000.0


def spmv_sketch_bytes(N, nnz, tw, p=8, pv=8):
    """Algorithmic HBM bytes of one SpMV + window-product + sketch launch (32-bit
    indices): values and column indices, row pointers, the input vector once
    (it is also the newest window vector and the sketched vector), the other
    tw - 1 window vectors, and the output vector."""
    return nnz * (pv + 4) + 4 * (N + 1) + p * N * (1 + max(tw - 1, 0) + 1)


def spmv_dia_sketch_bytes(N, ndiag, tw, p=8, pv=8):
    """The same for a matrix stored by diagonals: ndiag value streams of N
    entries (zero padding included), no index arrays, then the vectors.
    ndiag counts the streams the kernel reads: a diagonal found constant is
    passed to the kernel as a value and moves no bytes."""
    return ndiag * N * pv + p * N * (1 + max(tw - 1, 0) + 1)


def read_diagonals(h):
    """Value streams the step kernel reads: the stored diagonals less those
    found constant."""
    return len(h.spmv_layout()) - bin(h.const_diagonals()).count("1")


def update_bytes(N, tw, p=8):
    """One orthogonalisation update launch: read w, read tw window vectors, write w."""
    return p * N * (tw + 2)


KERNEL_SOURCES = ("paper_2311_14206_amd/csrc/sdr_kernels.hip",
                  "paper_2311_14206_amd/csrc/sdr_kernels.h",
                  "paper_2311_14206_amd/csrc/sdr_common.h")


def _strip_comments(src):
    """C/C++ source without comments and whitespace runs (string literals kept)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c == '"':
            j = i + 1
            while j < n and src[j] != '"':
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_digest():
    """Digest of the device sources, comments and layout ignored: HBM counters
    are valid for this digest only."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_summary_path(kernel_base, workload_name):
    return os.path.join(ROOT, "profiles", f"{kernel_base}_{workload_name}_hbm_traffic.md")


def read_traffic(path, kernel_key):
    """Calibrated HBM bytes per launch of kernel_key from a committed summary,
    or None if there is none or it was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    digest, value = None, None
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if ln.startswith("source_digest:"):
                digest = ln.split(":", 1)[1].strip()
            elif ln.startswith("traffic[") and ln.split("]", 1)[0][len("traffic["):] == kernel_key:
                value = float(ln.split("=", 1)[1])
    if digest != kernel_source_digest():
        return None
    return value


def _pmc_rows(path):
    out = collections.defaultdict(list)
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("sdr::", "").strip()
            out[name].append(float(r["Counter_Value"]))
    return out


def _rel_dir(path):
    """The directory of a profiler output file, as $R/... when under the repository."""
    d = os.path.dirname(os.path.abspath(path))
    rel = os.path.relpath(d, ROOT)
    return d if rel.startswith("..") else f"$R/{rel}"


def summarize_pmc(fetch_csv, write_csv, calib_mb, workload_name):
    """Markdown summary of two counter runs: per-kernel mean FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by the factor that maps the
    calibration copy's reading to its true size."""
    fetch, write = _pmc_rows(fetch_csv), _pmc_rows(write_csv)
    calib = calib_mb * (1 << 20)
    f_kib = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
    w_kib = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
    if f_kib <= 0 or w_kib <= 0:
        raise SystemExit("no calibration copy in the counter runs (run them with --copy-calib-mb)")
    ff, fw = calib / (1024.0 * f_kib), calib / (1024.0 * w_kib)
    R = "$R"
    run = (f"timeout -s KILL 240 rocprofv3 --pmc {{c}} --output-format csv -d {{d}} "
           f"-o run -- python3 {R}/bench.py --workload {workload_name} --steps 1 --warmup 0 "
           f"--no-cpu-baseline --no-extras --copy-calib-mb {calib_mb}")
    lines = [f"# HBM traffic per dispatch, {workload_name} solve (rocprofv3 counters)", "",
             "Commands (from /tmp with TMPDIR=/tmp; R is the repository root):", "",
             "    " + run.format(c="FETCH_SIZE", d=_rel_dir(fetch_csv)),
             "    " + run.format(c="WRITE_SIZE", d=_rel_dir(write_csv)),
             f"    python3 {R}/bench.py --summarize-pmc {_rel_dir(fetch_csv)}/{os.path.basename(fetch_csv)} "
             f"{_rel_dir(write_csv)}/{os.path.basename(write_csv)} --copy-calib-mb {calib_mb} "
             f"--workload {workload_name}", "",
             f"Calibration: one device copy of {calib_mb} MiB ({calib} bytes read and written) reads "
             f"FETCH_SIZE {f_kib:.1f} KiB and WRITE_SIZE {w_kib:.1f} KiB, so bytes = "
             f"{ff:.4f} x 1024 x FETCH_SIZE and {fw:.4f} x 1024 x WRITE_SIZE.", "",
             "| kernel | dispatches | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) | read MB | written MB | total MB |",
             "|---|---|---|---|---|---|---|"]
    keys = sorted(set(fetch) & set(write), key=lambda k: -statistics.mean(fetch[k]) * len(fetch[k]))
    machine = []
    for k in keys:
        if k.startswith("__amd") or k.startswith("at::"):
            continue
        fk, wk = statistics.mean(fetch[k]), statistics.mean(write[k])
        rb, wb = ff * 1024.0 * fk, fw * 1024.0 * wk
        lines.append(f"| {k} | {len(fetch[k])} | {fk:.1f} | {wk:.1f} | {rb / 1e6:.2f} | {wb / 1e6:.2f} | "
                     f"{(rb + wb) / 1e6:.2f} |")
        machine.append(f"traffic[{k}] = {rb + wb:.0f}")
    lines += ["", "Per-launch HBM bytes (read + written), as bench.py reads them:", "",
              f"source_digest: {kernel_source_digest()}"] + machine
    return "\n".join(lines) + "\n"


def _step_periods(trace, k1n):
    """Median step period (start of the step kernel to its next start, within
    a cycle) and median gap before the step kernel (end of the previous
    first-stream kernel to its start) of a kernel trace."""
    import numpy as np
    starts = sorted(s_ for s_, e, n in trace if n == k1n)
    per = np.diff(np.array(starts, dtype=np.float64)) / 1e3
    per = per[per < 3 * np.median(per)]  # (cycle boundaries left out)
    first = sorted((s_, e, n) for s_, e, n in trace
                   if n == k1n or n.startswith(("k_update<", "k_ilu_", "k_dct_sketch<")))
    gaps = [(b[0] - a[1]) / 1e3 for a, b in zip(first, first[1:]) if b[2] == k1n and a[2] != k1n]
    return float(np.median(per)), float(np.median(gaps)) if gaps else 0.0


def _mblk_summary(trace):
    """Median durations of the several-workgroup block least-squares kernels
    and of a whole block (step headers to finish), or '' without them."""
    import numpy as np
    names = ("k_mblk_head", "k_mblk_proj", "k_mblk_upd", "k_mblk_qr", "k_mblk_fin")
    ev = sorted((s_, e, n) for s_, e, n in trace if n.startswith(names))
    if not ev:
        return ""
    med = {}
    for nm in names:
        d = [(e - s_) / 1e3 for s_, e, n in ev if n.startswith(nm)]
        if d:
            med[nm] = float(np.median(d))
    blocks, cur = [], None
    for s_, e, n in ev:
        if n.startswith("k_mblk_head"):
            cur = s_
        elif n.startswith("k_mblk_fin") and cur is not None:
            blocks.append((e - cur) / 1e3)
            cur = None
    parts = ", ".join(f"{k[7:]} {v:.1f}" for k, v in med.items())
    return (f"Block least squares on several workgroups ({len(blocks)} blocks of up to 8 steps): median "
            f"kernel times (us) {parts}; a whole block, step headers to finish, median "
            f"{np.median(blocks):.1f} us.")


def summarize_kstats(stats_csv, trace_csv, bench_json, workload_name, flags="", plain_trace=None):
    """Markdown summary of a rocprofv3 kernel-trace run: per-kernel calls and
    durations, the step kernel's per-launch distribution, whether any of its
    launches overlapped a kernel of the least-squares stream, and the bench's
    own event timing of the same kernel.  With plain_trace (a kernel trace of
    the same command without --stats) also the step period of both runs."""
    import numpy as np

    def short(n):
        return n.split("(")[0].replace("void ", "").replace("sdr::", "")

    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    with open(trace_csv) as f:
        trace = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]))
                 for r in csv.DictReader(f)]
    with open(bench_json) as f:
        bj = json.loads(f.read().strip().splitlines()[-1])
    from workloads import WORKLOADS
    p = WORKLOADS[workload_name]
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    steps = [r for r in rows if short(r["Name"]).startswith(("k_spmv_dia_sketch<", "k_spmv_sketch<"))]
    k1 = max(steps, key=lambda r: float(r["TotalDurationNs"]))
    k1n = short(k1["Name"])
    d1 = sorted((s_, e) for s_, e, n in trace if n == k1n)
    dur = np.array([(e - s_) / 1e3 for s_, e in d1])
    side = sorted((s_, e) for s_, e, n in trace if n.startswith(("k_lsq_", "k_reduce_steps")))
    overlap = sum(1 for s_, e in d1 if any(a < e and b > s_ for a, b in side))
    R = "$R"
    kd = _rel_dir(stats_csv)
    sv = bj["solve"]
    prec_flag = (" --precision 1" if bj["config"].get("precision") == "mixed" else "") + \
        (" " + flags if flags else "")
    lines = [f"# rocprofv3 kernel statistics: GMRES-SDR solve, {workload_name} ({bj['dtype']})", "",
             f"Workload {bj['config']['workload']}; m = {p['m']}, k = {p['k']}, t = {p['t']}, "
             f"s = {p['s']}, zeta = {p['zeta']}, tol {p['tol']:g}; one solve from x0 = 0 with an empty "
             f"recycle space ({sv['iters']} Arnoldi steps, {sv['cycles']} cycles).", "",
             "Commands (from /tmp with TMPDIR=/tmp; R is the repository root):", "",
             f"    timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "
             f"{kd} -o run -- python3 {R}/bench.py --workload {workload_name}{prec_flag} --steps 1 "
             f"--warmup 0 --no-cpu-baseline --no-extras",
             f"    python3 {R}/bench.py --summarize-kstats {kd}/{os.path.basename(stats_csv)} "
             f"{_rel_dir(trace_csv)}/{os.path.basename(trace_csv)} BENCH.json --workload {workload_name}"
             + (f" --kstats-flags \"{flags}\"" if flags else "")
             + (f" --plain-trace {_rel_dir(plain_trace)}/{os.path.basename(plain_trace)}" if plain_trace else ""),
             "",
             f"(BENCH.json: the output line of `python3 bench.py --workload {workload_name}{prec_flag} "
             "--no-cpu-baseline --no-extras` run just before, on the same box.)", "",
             f"Kernel source digest (bench.py kernel_source_digest, comments ignored): {kernel_source_digest()}.",
             "",
             f"The step kernel {k1n} averages {float(k1['AverageNs']) / 1e3:.2f} us over {len(dur)} launches "
             f"here (median {np.median(dur):.2f} us, 5th and 95th percentiles "
             f"{np.percentile(dur, 5):.2f} and {np.percentile(dur, 95):.2f} us). "
             f"{overlap} of its launches overlapped a least-squares kernel of the second stream. "
             f"The bench's own HIP events (recorded by the dispatches themselves on sampled steps, "
             f"created without a system-scope fence) read {bj['roofline']['avg_us']:.2f} us over "
             f"{bj['arnoldi_step']['launches']} launches in the bench run.", ""]
    mb = _mblk_summary(trace)
    if mb:
        lines += [mb, ""]
    if plain_trace:
        with open(plain_trace) as f:
            ptrace = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]))
                      for r in csv.DictReader(f)]
        per_s, gap_s = _step_periods(trace, k1n)
        per_p, gap_p = _step_periods(ptrace, k1n)
        pd_ = _rel_dir(plain_trace)
        why = ": the statistics mode delays dispatches" if gap_s > gap_p + 0.5 else ""
        lines += [f"Step period (start of {k1n} to its next start within a cycle), median: "
                  f"{per_p:.2f} us in a kernel trace without --stats (median gap before the step kernel "
                  f"{gap_p:.2f} us), {per_s:.2f} us in the run above (gap {gap_s:.2f} us{why}). "
                  "The trace without --stats:", "",
                  f"    timeout -k 10 300 rocprofv3 --kernel-trace --output-format csv -d {pd_} -o run -- "
                  f"python3 {R}/bench.py --workload {workload_name}{prec_flag} --steps 1 --warmup 0 "
                  f"--no-cpu-baseline --no-extras", ""]
        mbp = _mblk_summary(ptrace)
        if mbp:
            lines += ["Without --stats: " + mbp, ""]
    lines += ["| Calls | Avg (us) | Total (ms) | % | Kernel |", "|---:|---:|---:|---:|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{100 * float(r['TotalDurationNs']) / total:.2f} | `{short(r['Name'])}` |")
    return "\n".join(lines) + "\n"


def _blas_threads():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return int(max([i.get("num_threads", 1) for i in info] or [1]))
    except Exception:  # pragma: no cover
        return 1


def cpu_baseline(A, b, p, gpu_iters):
    """The oracle's first two cycles of the same solve on the host: the first
    (no recycled block) once, the second (k recycled vectors, as every later
    cycle) per step for the remaining steps of the GPU solve."""
    from oracle import sdr_solve
    from oracle.sketch import sketch_operator
    blas_threads = _blas_threads()
    As = A.to_scipy()
    S = sketch_operator(A.n, p["s"], p["zeta"], p["s_seed"])
    kw = dict(m=p["m"], k=p["k"], t=p["t"], s=p["s"], zeta=p["zeta"], seed=p["s_seed"], tol=p["tol"], S=S)
    t0 = time.perf_counter()
    r1 = sdr_solve(As, b, max_cycles=1, **kw)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    r2 = sdr_solve(As, b, x0=r1.x, recycle=r1.recycle, max_cycles=1, **kw)
    t2 = time.perf_counter() - t0
    per_step2 = t2 / max(r2.iters, 1)
    value = t1 + per_step2 * max(gpu_iters - r1.iters, 0)
    return {"value": value, "unit": "s", "cores": int(blas_threads), "kind": "oracle",
            "sample": (f"the oracle's first two cycles of the same solve on the host: cycle 1 "
                       f"({r1.iters} steps, no recycled block) {t1:.1f} s, cycle 2 ({r2.iters} steps, "
                       f"k_hat = {r1.recycle.k}, the steady state of the later cycles) {t2:.1f} s = "
                       f"{per_step2 * 1e3:.1f} ms per step incl. its least squares, checks and "
                       f"eigen-step; extrapolated: cycle 1 + {gpu_iters - r1.iters} further steps at "
                       f"the cycle-2 rate (the GPU solve's {gpu_iters} steps); SciPy sparse products "
                       f"single-threaded, BLAS threads {blas_threads}, nproc {os.cpu_count()}")}


def _first_cycle_error(A, b, p, xg1):
    """Relative 2-norm error of a first-cycle x against the FP64 oracle's first
    cycle from x0 = 0 (and the oracle's time for it)."""
    import numpy as np
    from oracle import sdr_solve
    t0 = time.perf_counter()
    r = sdr_solve(A.to_scipy(), b, m=p["m"], k=p["k"], t=p["t"], s=p["s"], zeta=p["zeta"],
                  seed=p["s_seed"], tol=p["tol"], max_cycles=1)
    dt = time.perf_counter() - t0
    return [float(np.linalg.norm(x - r.x) / np.linalg.norm(r.x)) for x in xg1], dt


def _step_kernel_rate(kt, N, ndiag, p, pv):
    """Average duration and algorithmic bandwidth of the SpMV + sketch kernel
    from a handle's sampled kernel timings (diagonal storage)."""
    hist, launches = kt["window_hist"], kt["launches"]
    if not launches or kt["spmv_sketch_ms"] <= 0:
        return None
    byts = sum(hist[tw] * spmv_dia_sketch_bytes(N, ndiag, tw, p=p, pv=pv) for tw in range(len(hist)))
    sec = kt["spmv_sketch_ms"] * 1e-3
    return {"avg_us": 1e6 * sec / launches, "gbs": byts / sec / 1e9,
            "frac": byts / sec / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": byts / launches,
            "launches": launches}


def sequence_bench(dev, with_oracle=True):
    """The 20-system 3D sequence in FP64 and with the FP32 basis."""
    import numpy as np
    import torch
    from paper_2311_14206_amd.sdr import SDRSolver
    from workloads import workload, sequence_system, describe

    name = "cd3d_128_seq"
    A0, _, p = workload(name)
    systems = [sequence_system(A0, p, i) for i in range(1, p["n_systems"] + 1)]
    rp = torch.from_numpy(A0.row_ptr).to(dev)
    ci = torch.from_numpy(A0.col_idx).to(dev)
    vals = [torch.from_numpy(Ai.values).to(dev) for Ai, _ in systems]
    bs = [torch.from_numpy(bi).to(dev) for _, bi in systems]
    out = {"workload": describe(name), "m": p["m"], "k": p["k"], "t": p["t"], "s": p["s"],
           "tol": p["tol"], "variant": "exact (S A_i U recomputed per system)",
           "fp64_no_carry_note": "the same systems with the recycle space dropped before each "
                                 "(deflated restarting within a solve only), for comparison"}
    first = {}
    runs = ((0, "fp64", True), (1, "fp32_basis", True), (0, "fp64_no_carry", False))
    for prec, key, carry in runs:
        h = SDRSolver(rp, ci, vals[0], m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"],
                      zeta=p["zeta"], precision=prec, kernel_timing=64)
        # warm-up: one solve of system 1, then the recycle space is dropped
        h.solve(bs[0], tol=p["tol"])
        h.reset()
        h.kernel_times()
        torch.cuda.synchronize()
        xs, sts = [], []
        t0 = time.perf_counter()
        for i in range(len(systems)):
            if not carry:
                h.reset()  # deflated restarting within each solve only
            h.update_matrix(vals[i])
            x, st = h.solve(bs[i], tol=p["tol"])
            xs.append(x)
            sts.append(st)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        kt = h.kernel_times()
        relres = []
        for (Ai, bi), x in zip(systems, xs):
            xh = x.cpu().numpy()
            relres.append(float(np.linalg.norm(bi - Ai.to_scipy() @ xh) / np.linalg.norm(bi)))
        iters = [st["iters"] for st in sts]
        rate = _step_kernel_rate(kt, A0.n, read_diagonals(h), 8 if prec == 0 else 4,
                                 8 if prec == 0 else 4)
        out[key] = {"solves_per_s": len(systems) / total, "seconds_total": total,
                    "steps_per_system": iters, "steps_system1": iters[0],
                    "steps_mean_later": float(np.mean(iters[1:])),
                    "matvecs_total": int(sum(st["matvecs"] for st in sts)),
                    "converged_all": all(st["converged"] for st in sts),
                    "relres_host_max": max(relres),
                    "host_eig_seconds_total": float(sum(st["host_eig_seconds"] for st in sts)),
                    "step_kernel": rate}
        print(f"[bench] sequence {key}: {len(systems) / total:.2f} solves/s, steps {iters}, "
              f"max host relres {max(relres):.2e}", file=sys.stderr, flush=True)
        if not carry:
            h.close()
            continue
        # first cycle of system 1 on a fresh handle, for the error against the oracle
        h1 = SDRSolver(rp, ci, vals[0], m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"],
                       zeta=p["zeta"], precision=prec, max_cycles=1)
        x1, _ = h1.solve(bs[0], tol=p["tol"])
        first[key] = x1.cpu().numpy()
        h.close()
        h1.close()
        del xs
    if with_oracle:
        errs, dt = _first_cycle_error(systems[0][0], systems[0][1], p, [first["fp64"], first["fp32_basis"]])
        out["fp64"]["first_cycle_x_err_vs_oracle"] = errs[0]
        out["fp32_basis"]["first_cycle_x_err_vs_oracle"] = errs[1]
        out["oracle_first_cycle_seconds"] = dt
    return out


FP64_VALU_GOPS = 256 * 64 * 2.4  # FP64 vector lane-operations per ns: 78.6 TFLOP/s counts an FMA as 2


def srdct_bench(dev, with_oracle=True, reps=2):
    """The 1024^2 solve with the subsampled randomised DCT sketch (Section 6)."""
    import numpy as np
    import torch
    from paper_2311_14206_amd.sdr import SDRSolver
    from workloads import workload, describe

    name = "cd2d_1024"
    A, b, p = workload(name)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    vals = torch.from_numpy(A.values).to(dev)
    bd = torch.from_numpy(b).to(dev)
    h = SDRSolver(rp, ci, vals, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"], sketch=1,
                  kernel_timing=64)
    h.solve(bd, tol=p["tol"])  # warm-up
    h.kernel_times()
    times, st, x = [], None, None
    for _ in range(reps):
        h.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = h.solve(bd, tol=p["tol"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    kt = h.kernel_times()
    xh = x.cpu().numpy()
    relres = float(np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b))
    n_l = max(kt["launches"], 1)
    dct_us = 1e3 * kt["dct_sketch_ms"] / n_l
    # per entry and kept row: one multiply-add and the rotation's two
    # multiplies and two multiply-adds, FP64 lane operations
    ops = 5.0 * p["s"] * A.n
    out = {"workload": describe(name) + ", subsampled randomised DCT sketch",
           "time_to_tol_s": statistics.median(times), "times": times, "iters": st["iters"],
           "cycles": st["cycles"], "converged": st["converged"], "relres_host": relres,
           "dct_kernel": {"avg_us": dct_us, "bound": "alu",
                          "achieved_gops": ops / (dct_us * 1e3) if dct_us > 0 else None,
                          "peak_gops": FP64_VALU_GOPS,
                          "frac": ops / (dct_us * 1e3) / FP64_VALU_GOPS if dct_us > 0 else None,
                          "ops_per_launch": ops, "launches": kt["launches"]},
           "spmv_avg_us": 1e3 * kt["spmv_sketch_ms"] / n_l, "step_avg_us": 1e3 * kt["step_ms"] / n_l}
    print(f"[bench] DCT sketch: {statistics.median(times):.3f} s, {st['iters']} steps, DCT kernel "
          f"{dct_us:.1f} us, relres {relres:.2e}", file=sys.stderr, flush=True)
    h1 = SDRSolver(rp, ci, vals, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"], sketch=1,
                   max_cycles=1)
    x1, _ = h1.solve(bd, tol=p["tol"])
    x1 = x1.cpu().numpy()
    h.close()
    h1.close()
    if with_oracle:
        from oracle import sdr_solve
        t0 = time.perf_counter()
        r = sdr_solve(A.to_scipy(), b, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"],
                      tol=p["tol"], max_cycles=1, sketch="srdct")
        out["oracle_first_cycle_seconds"] = time.perf_counter() - t0
        out["first_cycle_x_err_vs_oracle"] = float(np.linalg.norm(x1 - r.x) / np.linalg.norm(r.x))
    return out


def helmholtz_bench(dev, with_oracle=True, reps=2):
    """The complex Helmholtz system in complex128 and with the complex64 basis."""
    import numpy as np
    import torch
    from paper_2311_14206_amd.sdr import SDRSolver
    from workloads import workload, describe

    name = "helmholtz_1024"
    A, b, p = workload(name)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    vals = torch.from_numpy(A.values).to(dev)
    bd = torch.from_numpy(b).to(dev)
    out = {"workload": describe(name), "m": p["m"], "k": p["k"], "t": p["t"], "s": p["s"], "tol": p["tol"]}
    first = {}
    for prec, key in ((0, "c128"), (1, "c64_basis")):
        h = SDRSolver(rp, ci, vals, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"],
                      zeta=p["zeta"], precision=prec, kernel_timing=64)
        h.solve(bd, tol=p["tol"])  # warm-up
        h.kernel_times()
        times, st, x = [], None, None
        for _ in range(reps):
            h.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = h.solve(bd, tol=p["tol"])
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        kt = h.kernel_times()
        xh = x.cpu().numpy()
        relres = float(np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b))
        rate = _step_kernel_rate(kt, A.n, read_diagonals(h), 16 if prec == 0 else 8,
                                 16 if prec == 0 else 8)
        out[key] = {"time_to_tol_s": statistics.median(times), "times": times, "iters": st["iters"],
                    "cycles": st["cycles"], "res_checks": st["res_checks"], "converged": st["converged"],
                    "relres_host": relres, "host_eig_seconds": st["host_eig_seconds"],
                    "host_eig_seconds_per_cycle": st["host_eig_seconds"] / max(st["cycles"], 1),
                    "step_kernel": rate}
        print(f"[bench] helmholtz {key}: {statistics.median(times):.3f} s, {st['iters']} steps, "
              f"{st['cycles']} cycles, host eig {st['host_eig_seconds']:.3f} s, relres {relres:.2e}",
              file=sys.stderr, flush=True)
        h1 = SDRSolver(rp, ci, vals, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"],
                       zeta=p["zeta"], precision=prec, max_cycles=1)
        x1, _ = h1.solve(bd, tol=p["tol"])
        first[key] = x1.cpu().numpy()
        h.close()
        h1.close()
    if with_oracle:
        errs, dt = _first_cycle_error(A, b, p, [first["c128"], first["c64_basis"]])
        out["c128"]["first_cycle_x_err_vs_oracle"] = errs[0]
        out["c64_basis"]["first_cycle_x_err_vs_oracle"] = errs[1]
        out["oracle_first_cycle_seconds"] = dt
    return out


def ilu_bench(dev, reps=2):
    """The 1024^2 convection-diffusion system right-preconditioned by ILU(0)
    (multicolour order): time to 1e-8 and the cost of one M^-1 apply.  The
    oracle's ILU(0) is pure Python, too slow at this size: its parity is held
    by the GPU tests at small sizes."""
    import numpy as np
    import torch
    from paper_2311_14206_amd.sdr import SDRSolver
    from workloads import workload, describe

    name = "cd2d_1024"
    A, b, p = workload(name)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    vals = torch.from_numpy(A.values).to(dev)
    bd = torch.from_numpy(b).to(dev)
    h = SDRSolver(rp, ci, vals, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"], zeta=p["zeta"],
                  precond=2, kernel_timing=64)
    h.solve(bd, tol=p["tol"])  # warm-up (and the factorisation)
    times, st, x = [], None, None
    for _ in range(reps):
        h.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = h.solve(bd, tol=p["tol"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    xh = x.cpu().numpy()
    relres = float(np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b))
    # one apply z = M^-1 v, timed alone
    z = h.precond_apply(bd)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nrep = 20
    e0.record()
    for _ in range(nrep):
        z = h.precond_apply(bd)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nrep
    # algorithmic bytes of one apply (two colours, packed factors): every
    # off-diagonal factor entry once (column index and value); per row its
    # position in the colour order, the input, 1/u_ii and z written; the
    # neighbours' values once (in for the first colour's rows, z for the
    # second's)
    n, nnz, ev = A.n, A.nnz, 8
    bytes_apply = (nnz - n) * (4 + ev) + n * (4 + ev + ev + ev) + n * ev
    out = {"workload": describe(name) + ", right ILU(0), multicolour order", "m": p["m"], "k": p["k"],
           "t": p["t"], "s": p["s"], "tol": p["tol"],
           "time_to_tol_s": statistics.median(times), "times": times, "iters": st["iters"],
           "cycles": st["cycles"], "converged": st["converged"], "relres_host": relres,
           "apply": {"ms": ms, "bytes": bytes_apply, "achieved_gbs": bytes_apply / (ms * 1e-3) / 1e9,
                     "peak_gbs": 8000.0, "launches": 2,
                     "note": "20 applies back to back timed with events (launch gaps included)"}}
    print(f"[bench] ilu(0) cd2d_1024: {statistics.median(times):.3f} s, {st['iters']} steps, "
          f"{st['cycles']} cycles, relres {relres:.2e}, apply {ms * 1e3:.1f} us", file=sys.stderr, flush=True)
    h.close()
    return out


def differentiated_bench(dev):
    """The differentiated solve on the theta-weighted 512^2 convection-diffusion
    operator: gradient-descent steps on ||x(theta) - x_t||^2, each a forward
    and an adjoint GMRES-SDR solve (the adjoint's recycle space carried from
    step to step, S A^T U recomputed for each theta) plus the gradient kernel.
    Reports seconds per gradient step, the Arnoldi steps and matrix-vector
    products of both solves, and the gradient at the final theta against a
    sparse direct solve (SuperLU factors of A(theta), solves with A and A^T)."""
    import numpy as np
    import scipy.sparse.linalg as spl
    import torch
    from paper_2311_14206_amd.autograd import sdr_solve as solve_ad
    from paper_2311_14206_amd.sdr import SDRSolver
    from workloads import describe, edge_weighted, randn, workload

    name = "cd2d_512_theta"
    A, b, p = workload(name)
    A0, theta0 = p["A0"], p["theta"]
    xt = randn(A.n, p["xt_seed"])

    def dv(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    h = SDRSolver(dv(A.row_ptr), dv(A.col_idx), dv(A.values), m=p["m"], k=p["k"], t=p["t"], s=p["s"],
                  seed=p["s_seed"], zeta=p["zeta"])
    rows = np.repeat(np.arange(A0.n), np.diff(A0.row_ptr))
    on = rows == A0.col_idx
    a0, offm = dv(A0.values), dv((~on).astype(np.float64))
    rows_t, diag_pos = dv(rows.astype(np.int64)), dv(np.nonzero(on)[0].astype(np.int64))

    def values_of(theta):
        """The edge-weighted entries of the workload as a torch function of theta:
        theta_e a_e off the diagonal, a_ii + sum_j (1 - theta_ij) a_ij on it."""
        shift = torch.zeros(A0.n, dtype=a0.dtype, device=a0.device).index_add(
            0, rows_t, (a0 - theta * a0) * offm)
        return theta * a0 * offm + a0 * (1 - offm) + torch.zeros_like(a0).index_add(0, diag_pos, shift)

    tol = p["tol"]
    bb, xtd = dv(b), dv(xt)

    def grad_step(th):
        x = solve_ad(values_of(th), bb, h, tol)
        loss = torch.sum((x - xtd) ** 2)
        loss.backward()
        return float(loss.detach())

    warm = dv(theta0).requires_grad_(True)
    grad_step(warm)  # warm-up, then both recycle spaces dropped
    h.reset()
    th = dv(theta0).requires_grad_(True)
    losses, times, fw, ad = [], [], [], []
    eta = None
    for _ in range(p["gd_steps"]):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses.append(grad_step(th))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        fw.append(h.last_forward_stats)
        ad.append(h.last_adjoint_stats)
        with torch.no_grad():
            if eta is None:
                eta = 1e-3 / float(th.grad.abs().max())
            th -= eta * th.grad
        th.grad = None
    # the gradient at the final theta against the sparse direct one
    th_np = th.detach().cpu().numpy()
    thr = dv(th_np).requires_grad_(True)
    loss_f = grad_step(thr)
    g = thr.grad.detach().cpu().numpy()
    lu = spl.splu(edge_weighted(A0, th_np).to_scipy().tocsc())
    xr = lu.solve(b)
    lam = lu.solve(2.0 * (xr - xt), trans="T")
    gr = np.where(on, 0.0, A0.values * (-lam[rows] * xr[A0.col_idx] + lam[rows] * xr[rows]))
    lr = float(np.sum((xr - xt) ** 2))
    gerr = float(np.linalg.norm(g - gr) / np.linalg.norm(gr))
    out = {"workload": describe(name) + f", x_t~N(0,1) seed {p['xt_seed']}; loss ||x(theta) - x_t||^2",
           "m": p["m"], "k": p["k"], "t": p["t"], "s": p["s"], "tol": tol, "gd_steps": p["gd_steps"],
           "seconds_per_gradient_step": statistics.median(times),
           "seconds_total": sum(times),
           "forward_iters": [f["iters"] for f in fw], "adjoint_iters": [a["iters"] for a in ad],
           "forward_matvecs_total": sum(f["matvecs"] for f in fw),
           "adjoint_matvecs_total": sum(a["matvecs"] for a in ad),
           "loss_first": losses[0], "loss_last": losses[-1],
           "final_theta": {"loss": loss_f, "loss_direct": lr, "gradient_rel_err_vs_direct": gerr,
                           "reference": "SuperLU factors of A(theta): x and the adjoint from direct solves"}}
    print(f"[bench] differentiated cd2d_512: {statistics.median(times):.3f} s per gradient step, "
          f"loss {losses[0]:.4e} -> {losses[-1]:.4e}, adjoint steps {ad[0]['iters']} ... {ad[-1]['iters']}, "
          f"gradient error vs direct {gerr:.1e}", file=sys.stderr, flush=True)
    h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cd2d_1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sequence and Helmholtz measurements (profiling runs)")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--sketch", type=int, default=0,
                    help="0: sparse sign; 1: subsampled randomised DCT (profiling runs)")
    ap.add_argument("--kstats-flags", default="",
                    help="with --summarize-kstats: the bench options of the profiled run (--sketch 1, ...)")
    ap.add_argument("--plain-trace", default=None,
                    help="with --summarize-kstats: a kernel trace of the same run without --stats")
    ap.add_argument("--precond", type=int, default=0,
                    help="right preconditioning of the timed solve: 0 none, 1 Jacobi, 2 ILU(0)")
    ap.add_argument("--lsq-kernel", type=int, default=0,
                    help="least-squares kernel: 0 automatic, 1 block Gram-Schmidt, 2 one launch per step")
    ap.add_argument("--timing-every", type=int, default=64,
                    help="time the SpMV and update kernels of every n-th Arnoldi step with HIP "
                         "events (events between kernels cost launch gaps; 1 times all)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary of two rocprofv3 counter runs and exit")
    ap.add_argument("--summarize-kstats", nargs=3, metavar=("STATS_CSV", "TRACE_CSV", "BENCH_JSON"),
                    help="write the kernel-statistics summary of a rocprofv3 kernel-trace run and exit")
    args = ap.parse_args()
    if args.summarize_kstats:
        sys.stdout.write(summarize_kstats(*args.summarize_kstats, args.workload, args.kstats_flags,
                                          args.plain_trace))
        return
    if args.summarize_pmc:
        sys.stdout.write(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1],
                                       args.copy_calib_mb or 256, args.workload))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_14206_amd.sdr import SDRSolver
    from workloads import workload, describe

    dev = "cuda:0"
    A, b, p = workload(args.workload)
    N, nnz = A.n, A.nnz
    print(f"[bench] workload {args.workload}: N={N} nnz={nnz} m={p['m']} k={p['k']} "
          f"t={p['t']} s={p['s']}", file=sys.stderr, flush=True)
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    vals = torch.from_numpy(A.values).to(dev)
    bd = torch.from_numpy(b).to(dev)
    h = SDRSolver(rp, ci, vals, m=p["m"], k=p["k"], t=p["t"], s=p["s"], seed=p["s_seed"],
                  zeta=p["zeta"], kernel_timing=args.timing_every, precision=args.precision,
                  sketch=args.sketch, lsq_kernel=args.lsq_kernel, precond=args.precond)
    if args.copy_calib_mb:
        src = torch.ones(args.copy_calib_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(args.warmup):
        h.reset()
        x, st = h.solve(bd, tol=p["tol"])
        print(f"[bench] warmup {w}: {st['seconds']:.3f} s, iters {st['iters']}, "
              f"cycles {st['cycles']}", file=sys.stderr, flush=True)
    h.kernel_times()  # clear
    torch.cuda.synchronize()
    times, stats = [], []
    t_all = time.perf_counter()
    for i in range(args.steps):
        h.reset()
        t0 = time.perf_counter()
        x, st = h.solve(bd, tol=p["tol"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(st)
        print(f"[bench] step {i}: {times[-1]:.3f} s, iters {st['iters']}, cycles {st['cycles']}, "
              f"relres {st['relres']:.2e}, host eig {st['host_eig_seconds']:.3f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t_all
    kt = h.kernel_times()
    st = stats[-1]
    if not st["converged"]:
        print("[bench] solve did not converge", file=sys.stderr)
        sys.exit(1)
    # true residual on the host, outside the timed region
    xh = x.cpu().numpy()
    relres_host = float(np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b))

    hist = kt["window_hist"]
    launches = kt["launches"]
    pb = (8 if args.precision == 0 else 4) * (2 if A.values.dtype.kind == "c" else 1)
    layout = h.spmv_layout()
    cpx = A.values.dtype.kind == "c"
    tname = ("sdr::cx<double>" if cpx else "double") if args.precision == 0 else \
        ("sdr::cx<float>" if cpx else "float")
    if layout:
        # instantiation: <type, diagonals (0: any), window bound (2 for t <= 2, else 4),
        # threads (512 while 8 waves of FP64 sketch bins fit 64 KiB of LDS; else the
        # generic 256-thread one)
        cm = h.const_diagonals()
        if 8 * (p["s"] + 6) * 8 <= 64 * 1024:
            # (last parameter: the constant-diagonal instantiation)
            cmv = "true" if cm and len(layout) in (5, 7) and p["t"] <= 3 else "false"
            k1_key = (f"k_spmv_dia_sketch<{tname}, {len(layout) if len(layout) in (3, 5, 7, 9) else 0}, "
                      f"{2 if p['t'] <= 2 else 3 if p['t'] == 3 else 4}, 512, {cmv}>")
        else:
            k1_key = f"k_spmv_dia_sketch<{tname}, 0, 4, 256, false>"
        k1_bytes = sum(hist[tw] * spmv_dia_sketch_bytes(N, read_diagonals(h), tw, p=pb, pv=pb)
                       for tw in range(len(hist)))
        const_note = (f"; {bin(cm).count('1')} constant diagonals passed as values, their streams "
                      "not read nor counted") if cm else ""
        k1_name = (f"k_spmv_dia_sketch (stencil SpMV on {len(layout)} diagonals {layout} + "
                   f"truncation-window products + sparse-sign sketch of the input basis vector{const_note})")
    else:
        k1_key = f"k_spmv_sketch<{tname}>"
        k1_bytes = sum(hist[tw] * spmv_sketch_bytes(N, nnz, tw, p=pb, pv=pb) for tw in range(len(hist)))
        k1_name = ("k_spmv_sketch (CSR SpMV + truncation-window products + sparse-sign sketch "
                   "of the input basis vector)")
    k2_bytes = sum(hist[tw] * update_bytes(N, tw, p=pb) for tw in range(len(hist)))
    k1_s = kt["spmv_sketch_ms"] * 1e-3
    k2_s = kt["update_ms"] * 1e-3
    step_s = kt["step_ms"] * 1e-3
    k1_gbs = k1_bytes / k1_s / 1e9 if k1_s > 0 else None
    step_gbs = (k1_bytes + k2_bytes) / step_s / 1e9 if step_s > 0 else None
    kernels_gbs = (k1_bytes + k2_bytes) / (k1_s + k2_s) / 1e9 if k1_s + k2_s > 0 else None
    med = statistics.median(times)
    line = {
        "metric": METRIC,
        "value": med,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_all / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": (("c128" if cpx else "f64") if args.precision == 0 else
                  ("c64-basis/c128" if cpx else "f32-basis/f64")),
        "data": "synthetic",
        "config": {"workload": describe(args.workload) + {0: "", 1: ", right Jacobi preconditioning",
                                                          2: ", right ILU(0) preconditioning"}[args.precond],
                   "m": p["m"], "k": p["k"], "t": p["t"], "s": p["s"], "zeta": p["zeta"],
                   "tol": p["tol"], "precision": "fp64" if args.precision == 0 else "mixed"},
        "single_solves_per_s": 1.0 / med,
        "solve": {"cycles": st["cycles"], "iters": st["iters"], "matvecs": st["matvecs"],
                  "inner_products": st["inner_products"], "res_checks": st["res_checks"],
                  "relres": st["relres"], "relres_host_check": relres_host,
                  "host_eig_seconds": st["host_eig_seconds"]},
        "roofline": {"bound": "hbm",
                     "kernel": k1_name,
                     "note": ("effective bandwidth: algorithmic bytes / kernel time; the counters "
                              "behind traffic count L2 egress, and this step's ~100 MB working set "
                              "fits the 256 MB last-level cache, so part of it is served from there "
                              "(sequence.*.step_kernel measures the 3D sequence, whose per-step "
                              "working set does not fit)"),
                     "achieved": k1_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (k1_gbs / HBM_PEAK_GBS) if k1_gbs else None,
                     "traffic": read_traffic(traffic_summary_path(k1_key.split("<")[0], args.workload),
                                             k1_key),
                     "avg_us": 1e6 * k1_s / max(launches, 1),
                     "bytes_per_launch": k1_bytes / max(launches, 1),
                     "kernel_source_digest": kernel_source_digest()},
        "arnoldi_step": {"spmv_orth_sketch_gbs_kernels": kernels_gbs,
                         "spmv_orth_sketch_gbs_step": step_gbs,
                         "update_avg_us": 1e6 * k2_s / max(launches, 1),
                         "step_avg_us": 1e6 * step_s / max(launches, 1),
                         "bytes_per_step": (k1_bytes + k2_bytes) / max(launches, 1),
                         "launches": launches},
    }
    h.close()
    del x, bd, vals, ci, rp
    torch.cuda.empty_cache()
    if not args.no_extras:
        line["sequence"] = sequence_bench(dev, with_oracle=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
        line["helmholtz"] = helmholtz_bench(dev, with_oracle=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
        line["srdct"] = srdct_bench(dev, with_oracle=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
        line["ilu"] = ilu_bench(dev)
        torch.cuda.empty_cache()
        line["differentiated"] = differentiated_bench(dev)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(A, b, p, st["iters"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
