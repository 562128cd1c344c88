"""Benchmark: adaptive s-step CG solves on one MI355X.

A step is one complete solve (every outer block: matrix powers, Gram,
condition estimate and s_k choice, coordinate recurrence, recovery, true
residual) of the single-solve workload: 3-D 7-point Poisson on 128^3
(n = 2,097,152, nnz = 14,581,760, CSR FP64), b ~ U[-1,1] (seed 0), x_1 = 0,
Chebyshev basis on [Lanczos lambda_min, Gershgorin lambda_max], s_max = 10,
target relative residual 1e-12.  Inputs are resident in device memory before
the timed region.

Prints one JSON line: solves/s with p50/p99 latency, the roofline of the
dominant kernel (the matrix-powers pass: the bytes of the stored form it reads
/ HIP-event time, with the rocprofv3 counter traffic and the plain-CSR
"effective" figure beside it), the same for the passes on a matrix without
value tables (`roofline_plain`: the 2048^2 variable-coefficient diffusion
operator), the basis+Gram bandwidth, the 256-system batch workload
(`batch256`: systems/s, latency, one-at-a-time rate, worst residual), and the
CPU oracle (plain-FP64 mode) timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "solves/s + p99 latency at relres≤1e-10; basis+Gram HBM GB/s vs peak"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "mpk_pass_poisson3d_128.pmc.md")
PMC_SUMMARY_PLAIN = os.path.join(ROOT, "profiles", "mpk_pass_diffusion2048.pmc.md")
TRACE_SUMMARY = os.path.join(ROOT, "profiles", "solve_poisson3d_128.kernel_trace.md")
TRACE_SUMMARY_PLAIN = os.path.join(ROOT, "profiles", "mpk_pass_diffusion2048.kernel_trace.md")
# the matrix-powers kernel's source: its HBM counters are stale once these change
MPK_SOURCES = [os.path.join(ROOT, "paper_1701_03989_amd", "csrc", f)
               for f in ("spmv.hip", "common.h")]
COPY_BYTES = 1 << 30  # the calibration copy: 1 GiB read and 1 GiB written per launch

WORKLOADS = {
    "poisson3d_128": dict(N=128, s_max=10, tol=1e-12, basis="chebyshev"),
    "poisson3d_64": dict(N=64, s_max=10, tol=1e-12, basis="chebyshev"),
    "poisson3d_96": dict(N=96, s_max=10, tol=1e-12, basis="chebyshev"),
}


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def form_bytes(fmt: int, stored: int, n: int) -> float:
    """Bytes of A one matrix-powers pass reads in the stored form it uses (the
    library's accounting): in the slice-diagonal form a 16-bit code per row
    and per 64-row slice its count, 8 distances and 4-entry table; otherwise
    per SELL-64 entry 3 (value index + 16-bit offset), 10 (value + 16-bit
    offset) or 12 (value + 32-bit index), per slice its offset and width, and
    with value tables its 4-entry table."""
    from paper_1701_03989_amd import sscg

    if fmt & sscg.FMT_SDIA:
        nslices = (n + 63) // 64
        return 2.0 * 64 * nslices + (4.0 + 4.0 * 8 + 32.0) * nslices
    vt = bool(fmt & sscg.FMT_VTAB)
    c16 = bool(fmt & sscg.FMT_COL16)
    per_entry = 3.0 if vt else (10.0 if c16 else 12.0)
    nslices = (n + 63) // 64
    return per_entry * stored + (12.0 + (32.0 if vt else 0.0)) * nslices


def form_name(fmt: int) -> str:
    """The matrix-powers kernel and the stored form it reads, for format bits fmt."""
    from paper_1701_03989_amd import sscg

    if fmt & sscg.FMT_SDPAIR:
        return "k_mpk_sdp (matrix-powers pass), slice-diagonal form, two slices per wavefront"
    if fmt & sscg.FMT_SDIA:
        return "k_mpk (matrix-powers pass), slice-diagonal form"
    if fmt & sscg.FMT_VTAB:
        return "k_mpk (matrix-powers pass), value tables + 16-bit column offsets"
    if fmt & sscg.FMT_COL16:
        return "k_mpk (matrix-powers pass), FP64 values + 16-bit column offsets"
    return "k_mpk (matrix-powers pass), FP64 values + 32-bit column indices"


def traffic_from_profile(path=PMC_SUMMARY):
    """HBM bytes per matrix-powers launch from a committed rocprofv3 PMC
    summary, if it was taken on the current kernel source; else None."""
    try:
        lines = open(path).read().splitlines()
        d = json.loads(next(l for l in lines if l.startswith('{"source_sha256_16"')))
    except (OSError, ValueError, StopIteration):
        return None
    if d.get("source_sha256_16") != source_hash(MPK_SOURCES):
        return None
    return d.get("hbm_bytes_per_launch")


# ---------------------------------------------------------------- profile summaries
def _short(name: str) -> str:
    return name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]


def _counter_rows(path):
    import csv

    out = {}
    for r in csv.DictReader(open(path)):
        out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def summarize_pmc(d: str, cmd: str, plain: bool = False) -> None:
    """profiles/<pmc summary> from four rocprofv3 --pmc runs under d:
    pmc_FETCH_SIZE, pmc_WRITE_SIZE (bench.py, or bench.py --plain-passes-only
    when plain; matrix-powers launches only) and copy_FETCH_SIZE,
    copy_WRITE_SIZE (bench.py --copy-calibration).  Each counter is scaled by
    COPY_BYTES / (what it reads for the plain copy)."""
    f = {c: _counter_rows(os.path.join(d, f"pmc_{c}", "p_counter_collection.csv"))
         for c in ("FETCH_SIZE", "WRITE_SIZE")}
    cp = {c: _counter_rows(os.path.join(d, f"copy_{c}", "p_counter_collection.csv"))
          for c in ("FETCH_SIZE", "WRITE_SIZE")}
    scale = {}
    for c, rows in cp.items():
        v = [x for k, xs in rows.items() if "copyBuffer" in k for x in xs]
        scale[c] = COPY_BYTES / (float(np.median(v)) * 1024.0)
    title = ("variable-coefficient 2-D diffusion 2048^2 (no value tables), sscg_mpk s = 10"
             if plain else "3-D Poisson 128^3 (slice-diagonal form, two slices per wavefront), whole solves")
    lines = [f"# HBM traffic of the matrix-powers pass (k_mpk), {title}", "",
             "Commands (repo root, MI355X; `cd /tmp && export TMPDIR=/tmp` first, R = repo root):", ""]
    lines += ["    " + l for l in cmd.splitlines()]
    lines += ["", "Counters are KiB per dispatch.  Calibration: a plain 1 GiB device copy "
              "(torch copy_, bench.py --copy-calibration) reads "
              f"{COPY_BYTES / 1024 / scale['FETCH_SIZE']:.0f} KiB of FETCH_SIZE and "
              f"{COPY_BYTES / 1024 / scale['WRITE_SIZE']:.0f} KiB of WRITE_SIZE, so FETCH_SIZE "
              f"is scaled by {scale['FETCH_SIZE']:.3f} and WRITE_SIZE by {scale['WRITE_SIZE']:.3f}.  "
              "Launches that stood down after convergence (counters near 0) are left out.", "",
              "| variant | launches | FETCH KiB | WRITE KiB | HBM MB (scaled) |", "|---|---|---|---|---|"]
    tot_b, tot_n = 0.0, 0
    for k in sorted(f["FETCH_SIZE"]):
        if not k.startswith("k_mpk"):
            continue
        fe = np.array(f["FETCH_SIZE"][k])
        wr = np.array(f["WRITE_SIZE"].get(k, []))
        if len(wr) != len(fe):
            continue
        ran = fe > 0.01 * np.median(fe)
        if not ran.any():
            continue
        b = fe[ran] * 1024 * scale["FETCH_SIZE"] + wr[ran] * 1024 * scale["WRITE_SIZE"]
        tot_b += float(b.sum())
        tot_n += int(ran.sum())
        lines.append(f"| {k} | {int(ran.sum())} | {fe[ran].mean():.0f} | {wr[ran].mean():.0f} | "
                     f"{b.mean() / 1e6:.1f} |")
    per = tot_b / max(tot_n, 1)
    lines += ["", f"Average over all {tot_n} launches: {per / 1e6:.1f} MB of HBM traffic per launch.",
              "", "Machine-readable (bench.py reads this line; stale once the kernel source changes):",
              "", json.dumps({"source_sha256_16": source_hash(MPK_SOURCES),
                              "hbm_bytes_per_launch": per, "launches": tot_n,
                              "fetch_scale": scale["FETCH_SIZE"], "write_scale": scale["WRITE_SIZE"]})]
    out = PMC_SUMMARY_PLAIN if plain else PMC_SUMMARY
    open(out, "w").write("\n".join(lines) + "\n")
    print("wrote", out)


def summarize_trace(d: str, cmd: str) -> None:
    """profiles/<trace summary> from a rocprofv3 --kernel-trace --stats run under d."""
    import csv

    stats = list(csv.DictReader(open(os.path.join(d, "kt_kernel_stats.csv"))))
    trace = sorted(csv.DictReader(open(os.path.join(d, "kt_kernel_trace.csv"))),
                   key=lambda r: int(r["Start_Timestamp"]))
    lines = ["# Kernel trace: adaptive s-step CG solves, 3-D Poisson 128^3 (n = 2,097,152)", "",
             "Command (repo root, MI355X; `cd /tmp && export TMPDIR=/tmp` first, R = repo root):", "",
             "    " + cmd, "",
             "Chebyshev basis, s_max = 10, tol 1e-12; every solve takes 62 blocks of s = 10.",
             "rocprofv3 kernel statistics over the whole run (durations in microseconds):", "",
             "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.0f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    # one solve period of the uninstrumented timed region: from the second
    # solve's k_eps_star (end of its set-up) to the third's (needs --warmup >= 1)
    idx = [i for i, r in enumerate(trace) if "k_eps_star" in r["Kernel_Name"]]
    if len(idx) >= 3:
        seg = trace[idx[1]:idx[2]]
        t0, t1 = int(seg[0]["Start_Timestamp"]), int(seg[-1]["End_Timestamp"])
        q = {}
        for r in seg:
            q.setdefault(r["Queue_Id"], []).append(r)
        main = max(q, key=lambda k: sum("k_mpk" in r["Kernel_Name"] for r in q[k]))
        ms = q[main]
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in ms)
        gaps = {}
        for a, b in zip(ms, ms[1:]):
            key = (_short(a["Kernel_Name"]).split("<")[0], _short(b["Kernel_Name"]).split("<")[0])
            gaps.setdefault(key, []).append(int(b["Start_Timestamp"]) - int(a["End_Timestamp"]))
        lines += ["", f"One solve period without timing events (second timed solve, from the end of "
                  f"its set-up to the end of the next one's): {(t1 - t0) / 1e3:.0f} us; the launch stream is busy {busy / 1e3:.0f} us "
                  f"({100.0 * busy / (t1 - t0):.0f} %), the rest is idle time between its kernels:", "",
                  "| after | before | count | mean gap us | total us |", "|---|---|---|---|---|"]
        for (a, b), v in sorted(gaps.items(), key=lambda kv: -sum(kv[1]))[:10]:
            lines.append(f"| {a} | {b} | {len(v)} | {np.mean(v) / 1e3:.1f} | {sum(v) / 1e3:.0f} |")
        side = [r for k, rs in q.items() if k != main for r in rs]
        if side:
            sb = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in side)
            names = sorted({_short(r["Kernel_Name"]) for r in side})
            lines += ["", f"Second stream (validation of speculative blocks): {', '.join(names)}; "
                      f"busy {sb / 1e3:.0f} us, overlapped with the launch stream."]
    open(TRACE_SUMMARY, "w").write("\n".join(lines) + "\n")
    print("wrote", TRACE_SUMMARY)


def summarize_trace_batched(d: str, cmd: str, workload: str, out: str | None = None,
                            precision: str = "fp64") -> None:
    """profiles/<workload>.kernel_trace.md from a rocprofv3 --kernel-trace --stats run
    of bench.py --workload batch256|serve under d: the kernels of the batched
    blocks (per graph replay) and those of the one-at-a-time baseline."""
    import csv
    import glob

    f = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    stats = list(csv.DictReader(open(f)))
    replays = sum(int(r["Calls"]) for r in stats if "k_batch_plan" in r["Name"])
    batched = [r for r in stats if "_batch" in r["Name"] or "k_batch" in r["Name"]]
    single = [r for r in stats if r not in batched and ("k_" in r["Name"])]
    title = {"batch256": "a batch of 256 uneven systems (11.6 M rows; adaptive Chebyshev s_max = "
                         "8, tol 1e-10), batched and one at a time",
             "serve": "the serving trace (200 requests, Poisson arrivals 200/s, operators of "
                      "1e4-4e6 rows, tol 1e-6-1e-12), served and one at a time"}[workload]
    if precision == "variable":
        title += " (basis precision chosen per outer block in the batched path; FP64 one at a time)"
    lines = [f"# Kernel trace: {title}", "",
             "Command (repo root, MI355X; `cd /tmp && export TMPDIR=/tmp` first, R = repo root):",
             "", "    " + cmd, "",
             f"Batched blocks: {replays} graph replays (one outer block for every admitted "
             f"system each); durations in microseconds:", "",
             "| kernel | calls | avg us | per replay us | total ms |", "|---|---|---|---|---|"]
    tot = 0.0
    for r in sorted(batched, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        tot += t
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{t / 1e3 / max(replays, 1):.1f} | {t / 1e6:.1f} |")
    lines += ["", f"Sum per replay: {tot / 1e3 / max(replays, 1):.0f} us.", "",
              "One-at-a-time baseline (sscg_solve per system), largest totals:", "",
              "| kernel | calls | avg us | total ms |", "|---|---|---|---|"]
    for r in sorted(single, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} |")
    path = out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               f"{workload}.kernel_trace.md")
    open(path, "w").write("\n".join(lines) + "\n")
    print("wrote", path)


def summarize_trace_plain(d: str, cmd: str) -> None:
    """profiles/<plain trace summary> from a rocprofv3 --kernel-trace --stats run
    of bench.py --plain-passes-only under d."""
    import csv

    stats = list(csv.DictReader(open(os.path.join(d, "kt_kernel_stats.csv"))))
    lines = ["# Kernel trace: matrix-powers passes on the variable-coefficient diffusion matrix",
             "", "2-D 5-point FV diffusion 2048^2 (n = 4,194,304, nnz = 20,963,328), log-normal "
             "coefficients (sigma 2, correlation length 16 cells, seed 0): every stored value "
             "distinct, so the pass reads FP64 values and 16-bit column offsets (10 bytes per "
             "entry).  sscg_mpk with s = 10 (two sequences, Chebyshev basis), repeated.", "",
             "Command (repo root, MI355X; `cd /tmp && export TMPDIR=/tmp` first, R = repo root):",
             "", "    " + cmd, "", "rocprofv3 kernel statistics (durations in microseconds):", "",
             "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.0f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    mpk = [r for r in stats if _short(r["Name"]).startswith("k_mpk")]
    calls = sum(int(r["Calls"]) for r in mpk)
    tot = sum(float(r["TotalDurationNs"]) for r in mpk)
    lines += ["", f"All k_mpk launches: {calls}, average {tot / max(calls, 1) / 1e3:.1f} us."]
    open(TRACE_SUMMARY_PLAIN, "w").write("\n".join(lines) + "\n")
    print("wrote", TRACE_SUMMARY_PLAIN)


def plain_passes(reps: int = 10, only: bool = False):
    """Matrix-powers passes on a matrix that keeps FP64 values (no value
    tables): sscg_mpk with s = 10, two sequences, Chebyshev basis on the
    matrix's estimated interval, on the variable-coefficient diffusion
    matrix 2048^2 (the mixed-precision workload's operator, not equilibrated),
    `reps` times; HIP events around each call's passes on the launch stream.
    Returns the roofline of those passes."""
    import torch

    from paper_1701_03989_amd import problems, sscg

    A, b, _ = problems.diffusion2d_system(2048, 0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Ad = sscg.DeviceCsr.from_host(A, dev)
    ctx = sscg.sscg_create(0)
    try:
        s = 10
        n = A.n
        ld = (n + 63) // 64 * 64
        rcol = s + 1
        lo, hi = sscg.sscg_spectral_bounds(ctx, Ad, 30, 0)
        Y = torch.zeros((2 * s + 1) * ld, dtype=torch.float64, device=dev)
        Y[:n] = torch.as_tensor(b, device=dev)
        Y[rcol * ld:rcol * ld + n] = torch.as_tensor(b[::-1].copy(), device=dev)
        fmt, stored = sscg.sscg_matrix_format(ctx, Ad)
        sscg.sscg_mpk(ctx, Ad, s, False, sscg.BASIS_CHEBYSHEV, lo, hi, Y, ld, rcol)  # warm-up
        torch.cuda.synchronize()
        if not only:
            sscg.sscg_set_timing(ctx, ["mpk"])
        for _ in range(reps):
            sscg.sscg_mpk(ctx, Ad, s, False, sscg.BASIS_CHEBYSHEV, lo, hi, Y, ld, rcol)
        torch.cuda.synchronize()
        if only:
            return None
        nl, ms, by = sscg.sscg_kernel_stats(ctx, "mpk")
        sscg.sscg_set_timing(ctx, False)
    finally:
        sscg.sscg_destroy(ctx)
    csr_extra = 12.0 * A.nnz + 4.0 * (n + 1) - form_bytes(fmt, stored, n)
    avg_ms = ms / max(nl, 1)
    alg = by / max(nl, 1)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    eff = (alg + csr_extra) / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(PMC_SUMMARY_PLAIN)
    return {
        "kernel": form_name(fmt),
        "workload": "diffusion2048 operator (n=4194304, nnz=20963328, variable coefficients), "
                    "sscg_mpk s=10, two sequences, Chebyshev",
        "format": {"col16": bool(fmt & sscg.FMT_COL16), "value_tables": bool(fmt & sscg.FMT_VTAB),
                   "stored_entries": int(stored)},
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
        "traffic_frac": (traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
        "effective_gbs": eff, "effective_frac": eff / HBM_PEAK_GBS,
        "algorithmic_bytes_per_launch": alg, "avg_launch_ms": avg_ms, "timed_launches": nl,
    }


def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info

        return max([int(d.get("num_threads", 1)) for d in threadpool_info()] + [1])
    except Exception:  # threadpoolctl missing or unreadable
        return 1


def cpu_baseline(A, b, x1, wl, gpu_blocks, budget_s=20.0):
    """The oracle (unchanged) on the same workload in its plain-FP64 mode
    (oracle.arith.Plain: scipy/numpy reductions, no correctly rounded sums,
    the timing mode; the correctly rounded mode is for parity only): its
    Chebyshev interval estimate, then outer blocks until about budget_s of CPU
    work; the solve time is extrapolated with the GPU's block count (same
    algorithm, same schedule of s = 10 blocks)."""
    from oracle import spectral, sstep
    from oracle.arith import Plain

    ar = Plain()
    t0 = time.perf_counter()
    lmin, lmax = spectral.chebyshev_interval(A, 30, 0, ar=ar)
    t_int = time.perf_counter() - t0
    # one block to size the sample, then one run of about budget_s
    opts = sstep.Opts(mode="adaptive", basis="chebyshev", s_max=wl["s_max"], tol=wl["tol"],
                      lmin=lmin, lmax=lmax, max_iters=1)
    t1 = time.perf_counter()
    res = sstep.solve(A, b, x1, opts, ar=ar)
    t_first = time.perf_counter() - t1
    # later blocks carry two sequences: about twice the first block's work
    nb = int(max(1, min(gpu_blocks, budget_s // max(2.0 * t_first, 1e-3))))
    if nb > 1:
        opts.max_iters = res.iters + (nb - 1) * wl["s_max"]
        t1 = time.perf_counter()
        res = sstep.solve(A, b, x1, opts, ar=ar)
        t_blocks = time.perf_counter() - t1
    else:
        t_blocks = t_first
    blocks = len(res.blocks)
    per_block = t_blocks / max(blocks, 1)
    t_solve = t_int + per_block * gpu_blocks
    threads = _blas_threads()
    # the first outer block again with one thread (a child process; the
    # interval estimate scaled by the same ratio)
    one = None
    code = ("import sys, time; sys.path.insert(0, %r); import numpy as np; "
            "from oracle import sstep; from oracle.arith import Plain; "
            "from paper_1701_03989_amd import problems; "
            "A, b, x1 = problems.poisson3d_128_system(0, N=%d); "
            "o = sstep.Opts(mode='adaptive', basis='chebyshev', s_max=%d, tol=%r, lmin=%r, "
            "lmax=%r, max_iters=1); t = time.perf_counter(); sstep.solve(A, b, x1, o, ar=Plain()); "
            "print(time.perf_counter() - t)") % (os.path.dirname(os.path.abspath(__file__)),
                                                  wl["N"], wl["s_max"], wl["tol"], lmin, lmax)
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300)
        t1b = float(r.stdout.strip().splitlines()[-1])
        ratio = t1b / max(t_first, 1e-9)
        one = {"value": 1.0 / (t_solve * ratio), "s_per_block": per_block * ratio,
               "sample": f"first outer block with one thread ({t1b:.2f} s vs {t_first:.2f} s with "
                         f"{threads}); the multi-threaded solve time scaled by that ratio"}
    except (OSError, ValueError, IndexError, subprocess.SubprocessError):
        one = None
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                     if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"plain-FP64 mode: Chebyshev interval estimate ({t_int:.2f} s) + first {blocks} "
                   f"outer blocks ({t_blocks:.2f} s, {per_block:.3f} s/block) of the same solve; "
                   f"solve time extrapolated to the GPU run's {gpu_blocks} blocks; cores = BLAS "
                   f"threads (the sparse products run on one)"),
        "single_core": one,
        "nproc": os.cpu_count(),
        "cpu_model": model,
    }


def run_batch(count: int, steps: int, warmup: int, precision: str = "fp64") -> dict:
    """The batch workload: uneven SPD systems (half Dirichlet Poisson 2-D/3-D,
    half shifted random graph Laplacians, sizes log-uniform in [1e3, 2e5]),
    adaptive s-step CG with the Chebyshev basis on each system's interval,
    s_max = 8, relres <= 1e-10 each.  A step is one batched solve of all
    systems (sscg_batch_solve); the same systems solved one at a time with
    sscg_solve are timed beside it (same algorithm, same FP64 results).  With
    precision 'variable' the batched solves pick each block's basis precision
    (FP32 where the rearranged eq. fb admits it); the one-at-a-time baseline
    stays FP64, and each batched result is compared with it."""
    import torch

    from oracle.arith import CR  # host check of the results only (not timed)
    from oracle.sstep import relres_of
    from paper_1701_03989_amd import problems, sscg

    t0 = time.perf_counter()
    systems = problems.batch_systems(count, seed=0)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    devA = [sscg.DeviceCsr.from_host(s.A, dev) for s in systems]
    bs = [torch.as_tensor(s.b, device=dev) for s in systems]
    xs = [torch.zeros(s.A.n, dtype=torch.float64, device=dev) for s in systems]
    lmin = [s.lmin for s in systems]
    lmax = [s.lmax for s in systems]
    opts = sscg.make_opts(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10,
                          precision=precision)
    ctx = sscg.sscg_create(0)
    hist = sscg.BatchHistory(len(systems), 4096)

    def batched():
        for x in xs:
            x.zero_()
        rc = sscg.sscg_batch_solve(ctx, devA, bs, xs, opts, lambda_min=lmin, lambda_max=lmax,
                                   hist=hist)
        assert rc == sscg.OK, f"batch status {rc}"

    # the first call of this batch shape times the launch-shape candidates
    # (sscg_set_batch_tuning) after its first blocks; later calls reuse the
    # choice
    for _ in range(warmup):
        batched()
        tuning = tuning if _ else sscg.sscg_batch_tuning(ctx)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        batched()
        lat.append(time.perf_counter() - ts)
        if warmup == 0 and _ == 0:
            tuning = sscg.sscg_batch_tuning(ctx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same timed calls with the untuned default shapes, for the tuner's gain
    sscg.sscg_set_batch_tuning(ctx, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batched()
    torch.cuda.synchronize()
    tuning["default_shapes_solves_per_s"] = len(systems) * steps / (time.perf_counter() - t0)
    sscg.sscg_set_batch_tuning(ctx, 1)
    # accuracy: true relative residuals recomputed on the host (correctly
    # rounded residual rows and sums)
    worst = 0.0
    ar = CR()
    for s, x in zip(systems, xs):
        xh = x.cpu().numpy()
        worst = max(worst, float(relres_of(ar, s.A, s.b, xh, ar.sqrt(ar.dot(s.b, s.b)))))
    blocks = hist.blocks.copy()
    nfp32 = int(sum(sum(hist.precisions(i)) for i in range(len(systems))))
    x_batched = [x.clone() for x in xs]
    # one at a time (FP64: the same systems and options; the same results
    # as a FP64 batch)
    h1 = sscg.History(4096, 8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for A_, b_, x_, s in zip(devA, bs, xs, systems):
        x_.zero_()
        o1 = sscg.make_opts(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10,
                            lmin=s.lmin, lmax=s.lmax)
        rc = sscg.sscg_solve(ctx, A_, b_, x_, o1, h1)
        assert rc == sscg.OK
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    err = [float(torch.linalg.norm(xb - x_) / torch.linalg.norm(x_)) for xb, x_ in
           zip(x_batched, xs)]
    sscg.sscg_destroy(ctx)
    nsys = len(systems)
    rows = sum(s.A.n for s in systems)
    nnz = sum(s.A.nnz for s in systems)
    return {
        "metric": "batched solves/s (systems per second) + p99 latency of a batch at relres<=1e-10",
        "value": nsys * steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"batch256: {nsys} SPD systems, rows log-uniform [1e3, 2e5] (total {rows}, "
                        f"nnz {nnz}), half Dirichlet Poisson 2-D/3-D, half graph Laplacians + "
                        f"1e-3*maxdeg*I, b~U[-1,1], x1=0",
            "method": "adaptive s-step CG (Alg. 4), batched launches, one block per graph replay",
            "basis": "chebyshev", "s_max": 8, "tol": 1e-10,
        },
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "worst_relres": worst,
        "max_blocks": int(blocks.max()),
        "graph_replays": int(hist.res.graph_launches),
        "tuning": tuning,
        "precision": precision,
        "fp32_blocks": nfp32,
        "blocks_total": int(blocks.sum()),
        "max_error_vs_fp64_one_at_a_time": max(err),
        "sequential_solves_per_s": nsys / t_seq,
        "speedup_vs_sequential": (nsys * steps / wall) / (nsys / t_seq),
        "generation_s": t_gen,
    }


def bench_batch(args) -> None:
    print(json.dumps(run_batch(args.batch_count, args.steps, args.warmup, args.precision)),
          flush=True)


def bench_precision(args) -> None:
    """Mixed precision against plain FP64 on one workload: the FP64 solve and
    the mixed solve (FP32 basis inside FP64 refinement) of the same system to
    the same tolerance, each timed over --steps solves; the error of the mixed
    solution against the FP64 one is reported with both true residuals."""
    import torch

    from paper_1701_03989_amd import problems, sscg

    if args.workload == "diffusion2048":
        A, b, x1 = problems.diffusion2d_system(2048, 0)
        kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10, equilibrate=True)
        desc = ("diffusion2048: variable-coefficient 2-D FV diffusion 2048^2, n=4194304, "
                "log-normal k (sigma 2, correlation length 16 cells, seed 0), b~U[-1,1], x1=0, "
                "equilibrated")
    else:
        wl = WORKLOADS[args.workload]
        A, b, x1 = problems.poisson3d_128_system(0, N=wl["N"])
        kw = dict(mode="adaptive", basis=wl["basis"], s_max=wl["s_max"], tol=wl["tol"])
        desc = f"{args.workload}: 3-D 7-point Poisson {wl['N']}^3, n={A.n}, b~U[-1,1] seed 0, x1=0"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Ad = sscg.DeviceCsr.from_host(A, dev)
    bd = torch.as_tensor(b, device=dev)
    x1d = torch.as_tensor(x1, device=dev)
    ctx = sscg.sscg_create(0)
    res = {}
    for prec in ("fp64", "mixed"):
        opts = sscg.make_opts(precision=prec, **kw)
        hist = sscg.History(1 << 16, kw["s_max"])
        xd = torch.empty_like(x1d)

        def one():
            xd.copy_(x1d)
            rc = sscg.sscg_solve(ctx, Ad, bd, xd, opts, hist)
            assert rc == sscg.OK, f"{prec} status {rc}"

        for _ in range(args.warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        x = xd.cpu().numpy()
        res[prec] = dict(solves_per_s=args.steps / wall, ms=wall / args.steps * 1e3, x=x,
                         relres=float(np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)),
                         iters=int(hist.res.iters), blocks=int(hist.res.blocks),
                         lam=[hist.res.lambda_min, hist.res.lambda_max])
    # the spectral estimate (30 Lanczos steps, Gershgorin) of the raw matrix; the solve's own
    # interval is that of the matrix it iterates on (equilibrated when equilibrating)
    raw_lo, raw_hi = sscg.sscg_spectral_bounds(ctx, Ad, 30, 0)
    sscg.sscg_destroy(ctx)
    xm, x64 = res["mixed"]["x"], res["fp64"]["x"]
    lam = res["fp64"]["lam"]
    out = {
        "metric": "solves/s at the target relres, mixed precision (FP32 basis, FP64 refinement) "
                  "vs plain FP64",
        "value": res["mixed"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["mixed"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 basis / f64 refinement",
        "data": "synthetic",
        "config": {"workload": desc, "method": "adaptive s-step CG (Alg. 4)", **kw},
        "fp64_solves_per_s": res["fp64"]["solves_per_s"],
        "speedup_vs_fp64": res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"],
        "relres_mixed": res["mixed"]["relres"],
        "relres_fp64": res["fp64"]["relres"],
        "error_mixed_vs_fp64": float(np.linalg.norm(xm - x64) / np.linalg.norm(x64)),
        "iters_mixed": res["mixed"]["iters"], "blocks_mixed": res["mixed"]["blocks"],
        "iters_fp64": res["fp64"]["iters"], "blocks_fp64": res["fp64"]["blocks"],
        "lambda": lam,
        "kappa_estimate": {"raw": raw_hi / raw_lo,
                           ("equilibrated" if kw.get("equilibrate") else "solved"): lam[1] / lam[0],
                           "method": "Gershgorin lambda_max / smallest Ritz value of 30 "
                                     "Lanczos steps"},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args) -> None:
    print(json.dumps(run_serve(args, args.precision)), flush=True)


def run_serve(args, precision: str) -> dict:
    """The serving workload: requests arrive as a Poisson process (rate
    --serve-rate per second, --serve-requests of them, seeded gaps); each asks
    for one SPD system drawn from a set of --serve-operators operators (sizes
    log-uniform in [1e4, 4e6], half Dirichlet Poisson, half shifted graph
    Laplacians), with its own right-hand side b ~ U[-1, 1] (seeded, drawn on the
    device) and a tolerance drawn from {1e-6, 1e-8, 1e-10, 1e-12}.  The server
    (continuous batching, admission by device-memory footprint) is timed from
    the first arrival; latency = completion - arrival.  The same requests served
    one at a time in arrival order by sscg_solve (FIFO, the measured solve
    times) give the baseline."""
    import torch

    from paper_1701_03989_amd import problems, sscg

    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    ops = problems.batch_systems(args.serve_operators, seed=100, nlo=1e4, nhi=4e6)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    devA = [sscg.DeviceCsr.from_host(s.A, dev) for s in ops]
    nreq = args.serve_requests
    arrive = np.cumsum(rng.exponential(1.0 / args.serve_rate, size=nreq))
    arrive -= arrive[0]
    which = rng.integers(0, len(ops), size=nreq)
    tols = rng.choice([1e-6, 1e-8, 1e-10, 1e-12], size=nreq)
    gen = torch.Generator(device=dev)
    bs = []
    for i in range(nreq):
        gen.manual_seed(1000 + i)
        n = ops[which[i]].A.n
        bs.append(torch.rand(n, dtype=torch.float64, device=dev, generator=gen) * 2.0 - 1.0)
    xs = [torch.zeros_like(b) for b in bs]
    opts = sscg.make_opts(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10,
                          precision=precision, max_iters=args.serve_max_iters)
    ctx = sscg.sscg_create(0)
    rows_needed = sum(((ops[w].A.n + 1023) // 1024) * 1024 for w in which)
    pool_rows = int(min(rows_needed, args.serve_pool_rows))
    pool_nnz = int(12 * pool_rows)
    srv = sscg.sscg_server_create(ctx, opts, pool_rows, pool_nnz, args.serve_slots)
    torch.cuda.synchronize()
    done_at = np.full(nreq, np.nan)
    status = np.full(nreq, -99)
    rid = {}
    pending = set()
    i = 0
    steps = 0
    start = time.perf_counter()
    while i < nreq or pending:
        now = time.perf_counter() - start
        while i < nreq and arrive[i] <= now:
            s = ops[which[i]]
            r = sscg.sscg_server_submit(ctx, srv, devA[which[i]], bs[i], xs[i], float(tols[i]),
                                        s.lmin, s.lmax)
            rid[r] = i
            pending.add(r)
            i += 1
        if not pending:
            time.sleep(max(0.0, arrive[i] - (time.perf_counter() - start)))
            continue
        run, q, ret = sscg.sscg_server_step(ctx, srv)
        steps += 1
        if ret or (run == 0 and q == 0):
            t = time.perf_counter() - start
            for r in list(pending):
                p = sscg.sscg_server_poll(ctx, srv, r)
                if p["state"] == 2:
                    # a tolerance below what the method attains ends in
                    # BREAKDOWN or NOT_CONVERGED (Algorithm 4 has no restart)
                    status[rid[r]] = p["status"]
                    done_at[rid[r]] = t
                    pending.discard(r)
    makespan = float(np.nanmax(done_at))
    lat = done_at - arrive
    occ = sscg.sscg_server_stats(ctx, srv)
    nfp32 = nblk = 0
    for r in rid:
        h = sscg.sscg_server_history(ctx, srv, r)
        nfp32 += sum(h["fp32"])
        nblk += len(h["s_k"])
    sscg.sscg_server_destroy(srv)
    # accuracy of every served result, recomputed in FP64 on the host
    worst = 0.0
    unmet = []
    for k in range(nreq):
        s = ops[which[k]]
        b = bs[k].cpu().numpy()
        x = xs[k].cpu().numpy()
        rel = float(np.linalg.norm(b - s.A.matvec(x)) / np.linalg.norm(b))
        if status[k] == sscg.OK:
            worst = max(worst, rel / tols[k])
        else:
            unmet.append({"request": k, "n": s.A.n, "operator": s.kind, "tol": float(tols[k]),
                          "status": int(status[k]), "relres": rel})
    met = int(np.sum(status == sscg.OK))
    x_served = [x.clone() for x in xs]
    # one at a time (FP64), first come first served, with the measured solve times
    h1 = sscg.History(8192, 8)
    clock, seq_lat = 0.0, []
    for k in range(nreq):
        s = ops[which[k]]
        xs[k].zero_()
        o1 = sscg.make_opts(mode="adaptive", basis="chebyshev", s_max=8, tol=float(tols[k]),
                            max_iters=args.serve_max_iters,
                            lmin=s.lmin, lmax=s.lmax)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        rc = sscg.sscg_solve(ctx, devA[which[k]], bs[k], xs[k], o1, h1)
        d = time.perf_counter() - ts
        if precision == "fp64":
            assert rc == status[k], (k, rc, status[k])  # the same bits as served
        clock = max(clock, arrive[k]) + d
        seq_lat.append(clock - arrive[k])
    err = [float(torch.linalg.norm(xv - x_) / torch.linalg.norm(x_)) for xv, x_ in
           zip(x_served, xs)]
    sscg.sscg_destroy(ctx)
    out = {
        "metric": "served solves/s + p50/p99 latency (arrival to result) at per-request relres",
        "value": met / makespan,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": makespan / max(steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"serve: {nreq} requests, Poisson arrivals {args.serve_rate}/s, "
                        f"{len(ops)} operators of {sum(s.A.n for s in ops)} rows in total "
                        f"(sizes log-uniform [1e4, 4e6]), tol in {{1e-6,1e-8,1e-10,1e-12}}",
            "method": "continuous batching of adaptive s-step CG (Alg. 4), one outer block per "
                      "step for all admitted systems",
            "basis": "chebyshev", "s_max": 8, "pool_rows": pool_rows, "slots": args.serve_slots,
            "max_iters": args.serve_max_iters,
        },
        "offered_rate": args.serve_rate,
        "replays": occ["replays"],
        "mean_rows_per_replay": occ["rows_active"] / max(occ["replays"], 1),
        "precision": precision,
        "fp32_blocks": nfp32,
        "blocks_total": nblk,
        "max_error_vs_fp64_one_at_a_time": max(err),
        "median_error_vs_fp64_one_at_a_time": float(np.median(err)),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "worst_relres_over_tol": worst,
        "requests_meeting_tol": met,
        "requests_unmet": unmet,
        "sequential_solves_per_s": met / max(clock, 1e-9),
        "sequential_p50_ms": float(np.percentile(seq_lat, 50) * 1e3),
        "sequential_p99_ms": float(np.percentile(seq_lat, 99) * 1e3),
        "generation_s": t_gen,
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson3d_128",
                    choices=sorted(WORKLOADS) + ["batch256", "serve", "diffusion2048"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "variable"],
                    help="mixed: time the mixed-precision solve against plain FP64; variable: "
                         "the batch256 / serve workloads with the basis precision chosen per "
                         "outer block, against FP64 one at a time")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="batch256 workload: number of systems")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="arrivals per second")
    ap.add_argument("--serve-operators", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-pool-rows", type=int, default=96 << 20)
    ap.add_argument("--serve-max-iters", type=int, default=20000,
                    help="iteration cap of every served and one-at-a-time solve (the largest "
                         "operator needs about 6900 at tol 1e-12)")
    ap.add_argument("--basis", choices=["chebyshev", "monomial", "newton"], default=None,
                    help="basis of the single-solve workloads (default: the workload's)")
    ap.add_argument("--c-mode", choices=["const", "theory"], default="const",
                    help="c_{k,j}: the constant 1, or 6 N_k j kappa(A) of Section 4.1")
    ap.add_argument("--forms", type=int, default=31,
                    help="compact forms of A the library may use (bits: 1 16-bit offsets, "
                         "2 value tables, 4 slice-diagonal, 8 slice-diagonal in pairs of "
                         "slices, 16 one value per distance; default all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-classical", action="store_true",
                    help="skip timing classical CG (s = 1) beside the s-step solve")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the plain-form passes and the batch256 object of the default run")
    ap.add_argument("--plain-passes-only", action="store_true",
                    help="only run the plain-form matrix-powers passes (for rocprofv3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="write the PMC summary under profiles/ from rocprofv3 runs in DIR")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write the kernel-trace summary under profiles/ from a rocprofv3 run in DIR")
    ap.add_argument("--summarize-pmc-plain", metavar="DIR",
                    help="the PMC summary of the plain-form passes (--plain-passes-only runs)")
    ap.add_argument("--summarize-trace-plain", metavar="DIR",
                    help="the kernel-trace summary of the plain-form passes")
    ap.add_argument("--profile-cmd", default="", help="the command(s) to quote in a summary")
    ap.add_argument("--summarize-trace-batched", metavar="DIR",
                    help="the kernel-trace summary of --workload batch256|serve")
    ap.add_argument("--summary-out", default=None, help="where to write that summary")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.profile_cmd)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.profile_cmd)
        return
    if args.summarize_pmc_plain:
        summarize_pmc(args.summarize_pmc_plain, args.profile_cmd, plain=True)
        return
    if args.summarize_trace_plain:
        summarize_trace_plain(args.summarize_trace_plain, args.profile_cmd)
        return
    if args.summarize_trace_batched:
        summarize_trace_batched(args.summarize_trace_batched, args.profile_cmd, args.workload,
                                args.summary_out, args.precision)
        return
    if args.plain_passes_only:
        plain_passes(reps=args.steps, only=True)
        return
    if args.copy_calibration:
        import torch

        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 8, "copies": 5}))
        return
    if args.precision == "variable" and args.workload not in ("batch256", "serve"):
        print("bench.py: --precision variable applies to the batch256 and serve workloads "
              "(batches and servers)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch256" and args.gpus == 1:
        bench_batch(args)
        return
    if args.workload == "serve" and args.gpus == 1:
        bench_serve(args)
        return
    if (args.precision == "mixed" or args.workload == "diffusion2048") and args.gpus == 1:
        bench_precision(args)
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding across GPUs is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1701_03989_amd import problems, sscg

    wl = dict(WORKLOADS[args.workload])
    variant = args.basis not in (None, wl["basis"]) or args.c_mode != "const" or args.forms != 31
    if args.basis:
        wl["basis"] = args.basis
    A, b, x1 = problems.poisson3d_128_system(0, N=wl["N"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Ad = sscg.DeviceCsr.from_host(A, dev)
    bd = torch.as_tensor(b, device=dev)
    x1d = torch.as_tensor(x1, device=dev)
    xd = torch.empty_like(x1d)
    opts = sscg.make_opts(mode="adaptive", basis=wl["basis"], s_max=wl["s_max"], tol=wl["tol"],
                          c_mode=args.c_mode)
    ctx = sscg.sscg_create(0)
    sscg.sscg_set_forms(ctx, args.forms)
    hist = sscg.History(4096, wl["s_max"])

    def one_solve():
        xd.copy_(x1d)
        rc = sscg.sscg_solve(ctx, Ad, bd, xd, opts, hist)
        assert rc == sscg.OK, f"solve status {rc}"

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    # timed region: K solves without instrumentation (an event record costs the
    # stream a few microseconds, which would show up in solves/s)
    sscg.sscg_set_timing(ctx, False)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        one_solve()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the returned x: true relative residual, recomputed independently in FP64
    x = xd.cpu().numpy()
    # the roofline kernel: the same K solves again, HIP events around every
    # matrix-powers launch on its own stream
    sscg.sscg_set_timing(ctx, ["mpk"])
    for _ in range(args.steps):
        one_solve()
    stats = {"mpk": sscg.sscg_kernel_stats(ctx, "mpk")}
    # per-family breakdown from one more solve with every family timed
    sscg.sscg_set_timing(ctx, True)
    one_solve()
    brk = {f: sscg.sscg_kernel_stats(ctx, f) for f in sscg.FAMILIES}
    sscg.sscg_set_timing(ctx, False)
    relres = float(np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b))
    # classical CG on the same system and tolerance: s_k = 1 in every block
    # (Section 4.2), through the same kernels; time to solution for context
    classical = None
    if not args.no_classical:
        oc = sscg.make_opts(mode="fixed", fixed_s=1, s_max=wl["s_max"], tol=wl["tol"])
        hc = sscg.History(1 << 14, wl["s_max"])
        xd.copy_(x1d)
        sscg.sscg_solve(ctx, Ad, bd, xd, oc, hc)  # warm-up
        kc = max(1, min(args.steps, 5))
        torch.cuda.synchronize()
        tc = time.perf_counter()
        for _ in range(kc):
            xd.copy_(x1d)
            rc = sscg.sscg_solve(ctx, Ad, bd, xd, oc, hc)
            assert rc == sscg.OK, f"classical CG status {rc}"
        torch.cuda.synchronize()
        wc = time.perf_counter() - tc
        xc = xd.cpu().numpy()
        classical = {
            "solves_per_s": kc / wc, "ms_per_solve": wc / kc * 1e3, "iters": int(hc.res.iters),
            "relres": float(np.linalg.norm(b - A.matvec(xc)) / np.linalg.norm(b)),
            "method": "Algorithm 2 with s = 1 (classical CG), same kernels and tolerance",
        }
    fmt, stored = sscg.sscg_matrix_format(ctx, Ad)
    sscg.sscg_destroy(ctx)

    n_mpk, ms_mpk, by_mpk = stats["mpk"]
    avg_ms = ms_mpk / max(n_mpk, 1)
    alg = by_mpk / max(n_mpk, 1)  # bytes of the stored form read + vectors
    mpk_gbs = alg / (avg_ms * 1e-3) / 1e9
    # the same passes priced at the plain CSR form (12 B per nonzero, 4 per row)
    csr_extra = 12.0 * A.nnz + 4.0 * (A.n + 1) - form_bytes(fmt, stored, A.n)
    eff_gbs = (alg + csr_extra) / (avg_ms * 1e-3) / 1e9
    bg_by = brk["mpk"][2] + brk["gram"][2]
    bg_ms = brk["mpk"][1] + brk["gram"][1]
    bg_gbs = bg_by / (bg_ms * 1e-3) / 1e9
    bg_eff = (bg_by + csr_extra * brk["mpk"][0]) / (bg_ms * 1e-3) / 1e9
    # the committed counters were taken on the default workload and options
    traffic = traffic_from_profile() if not variant and args.workload == "poisson3d_128" else None
    sched = hist.schedule
    out = {
        "metric": METRIC,
        "value": args.steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: 3-D 7-point Poisson {wl['N']}^3, n={A.n}, nnz={A.nnz}, "
                        f"b~U[-1,1] seed 0, x1=0",
            "method": "adaptive s-step CG (Alg. 4)",
            "basis": wl["basis"], "s_max": wl["s_max"], "tol": wl["tol"],
            "c": "6 N_k j kappa(A), kappa estimated" if args.c_mode == "theory" else 1.0,
        },
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "relres": relres,
        "blocks": hist.blocks,
        "iters": int(hist.res.iters),
        "schedule_head": sched[:12],
        "classical_cg": classical,
        "lambda": [hist.res.lambda_min, hist.res.lambda_max],
        "basis_gram_gbs": bg_gbs,
        "basis_gram_frac": bg_gbs / HBM_PEAK_GBS,
        "basis_gram_effective_frac": bg_eff / HBM_PEAK_GBS,
        "kernel_ms": {f: brk[f][1] / max(brk[f][0], 1) for f in brk},
        "kernel_launches_per_solve": {f: brk[f][0] for f in brk},
        "roofline": {
            "kernel": form_name(fmt),
            "bound": "hbm",
            "achieved": mpk_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": mpk_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_frac": (traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
            "traffic_note": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_note": "bytes of the stored form the pass reads (slice-diagonal form: "
                                "2 B per row + per-slice tables) + 8 B per vector element",
            "effective_gbs": eff_gbs,
            "effective_frac": eff_gbs / HBM_PEAK_GBS,
            "effective_note": "the same passes priced at plain CSR (12 B per nonzero + 4 B per "
                              "row): the problem's bytes, not moved bytes",
            "avg_launch_ms": avg_ms,
            "timed_launches": n_mpk,
        },
    }
    if not variant and args.workload == "poisson3d_128" and not args.no_extra:
        out["roofline_plain"] = plain_passes()
        out["batch256"] = run_batch(256, 3, 1)
        # serving with the basis precision chosen per outer block (the mixed
        # FP32/FP64 path) against FP64 one at a time
        out["serve"] = run_serve(args, "variable")
    if not args.no_cpu_baseline and not variant:
        out["cpu_baseline"] = cpu_baseline(A, b, x1, wl, hist.blocks, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
