"""Benchmark: Lennard-Jones pair interactions per second of the AICA hot path on one MI355X.

One step = one pass of the whole per-step path over one batch of synthetic input:
  aica_bin (locate, CSR occupancy, work list) + aica_forces + aica_forces_adjoint,
in FP32 pair arithmetic (compensated FP32 force sums, FP64 energy and virial).
The same step is also timed in FP64, and the forward alone in both precisions.
Molecules move between steps: every step bins its own position set x_k = x_0 + k delta
(delta a seeded displacement of about 0.005 sigma per coordinate, the distance an LJ fluid
at T* = 1 covers in one step of dt = 0.005), all sets resident in HBM before timing.

Prints ONE JSON line (rank 0).  `value` = (sum of npairs over the timed steps) / (timed
seconds) for the FP32 forward+adjoint step.  `roofline` is the dominant kernel's algorithmic
FLOP rate (HIP events on the stream the kernel runs on) against the FP32 vector
peak; `cpu_baseline` is the FP64 oracle timed on a bounded sample of rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LJ pair interactions/s (fwd, fwd+adjoint), FP32 vs FP64 GPU at stated error"
FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
GAMMA = 0.1                  # weight of U in the adjoint's loss L = sum G.F + gamma U
FP64_PEAK_TFLOPS = 78.6
# algorithmic FLOPs (FMA = 2, reciprocal = 1): forward per pair inside the cut-off, per rejected
# candidate (difference, squared distance, compare), adjoint per pair inside the cut-off
FLOP_FWD_PAIR, FLOP_REJECT, FLOP_ADJ_PAIR = 31, 8, 60


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from paper_cs_0702131_amd import workloads as W
    if name == "channel":
        return W.config5()
    if name == "binary":
        return W.config4()
    if name == "random":
        return W.config2()
    if name == "fcc864":
        return W.config1()
    if name.startswith("channel@"):
        return W.config5(scale=float(name.split("@")[1]))
    if name == "wedge":  # rotating referral: one of 12 sectors of an annulus, periodic in z
        return W.wedge(seed=16, r0=100.0, r1=200.0, n_sectors=12, Lz=60.0, nr=83, nphi=90, nz=50, density=0.8)
    raise SystemExit(f"unknown workload {name}")


# Kernel sources whose digest ties the traffic counters to the code they were measured on.
KERNEL_SOURCES = ["aica_pair.inc", "aica_adjoint_pair.inc", "aica_device.hip", "aica_kernels.h", "aica_adjoint.inc"]


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_cs_0702131_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


COUNTERS_FILE = "counters_pair_{workload}_fp32.txt"


def measured_counters(kernel, workload):
    """Per-launch figures of a pair kernel ("pair_fwd" / "pair_adj") from the committed counter summary of
    `workload`: HBM traffic in bytes (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration),
    VALU issue as a fraction of the chip's issue peak, and executed VALU FLOPs.  Empty when the summary is
    missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", COUNTERS_FILE.format(workload=workload))
    if not os.path.exists(path):
        return {}
    out, digest = {}, None
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) >= 2 and f[0] == "sources_sha256:":
                digest = f[1]
            elif len(f) == 6 and f[0] == "traffic:" and f[1] == kernel:
                out["traffic"] = float(f[2]) * 1024 * float(f[3]) + float(f[4]) * 1024 * float(f[5])
            elif len(f) == 3 and f[0] == "issue:" and f[1] == kernel:
                out["valu_issue_frac"] = float(f[2])
            elif len(f) == 3 and f[0] == "flops:" and f[1] == kernel:
                out["executed_flop"] = float(f[2])
    return out if digest == kernel_digest() else {}


PAIR_KERNELS = {"pair_fwd": "k_pair<float, 0, 0, true, false>", "pair_adj": "k_pair_adj<float, 0, false>"}
TIMERS = ("pair_fwd", "pair_adj", "bin", "finalize", "finalize_adj")


def moving_sets(wl, count, step=0.005, seed=11):
    """Positions of `count` consecutive steps, x_k = x_0 + k delta with delta ~ N(0, step) per coordinate
    (seeded), rounded to the position grid, wrapped on periodic axes and reflected at walls.  With rotating
    referral only the axis periodic by translation (z) moves."""
    from paper_cs_0702131_amd import workloads as W
    delta = np.random.default_rng(seed).normal(0.0, step, size=wl.x.shape)
    lo, hi = np.asarray(wl.mesh.lo, float), np.asarray(wl.mesh.hi, float)
    periodic = set(wl.periodic_axes)
    if wl.rotations is not None:
        delta[:, :2] = 0.0
        periodic = {2}
    sets = [wl.x]
    for k in range(1, count):
        x = wl.x + k * delta
        for a in range(3):
            if a in periodic:
                x[:, a] = lo[a] + np.mod(x[:, a] - lo[a], hi[a] - lo[a])
            else:
                x[:, a] = np.where(x[:, a] < lo[a], 2 * lo[a] - x[:, a], x[:, a])
                x[:, a] = np.where(x[:, a] > hi[a], 2 * hi[a] - x[:, a], x[:, a])
        x = W.qround(x)
        for a in range(3):
            if a in periodic:
                x[:, a] = np.where(x[:, a] >= hi[a], x[:, a] - (hi[a] - lo[a]), x[:, a])
            x[:, a] = np.clip(x[:, a], lo[a], hi[a])
        sets.append(x)
    return sets


def timed_steps(A, d, xs, sp, wl, G, precision, steps, warmup, adjoint=True):
    """Warm-up steps on xs[0 .. warmup-1], then `steps` timed steps on xs[warmup ..], each binning its own
    position set.  Returns the time, the per-kernel timers, npairs of every timed step and the routes by which
    each timed binning located its molecules."""
    import torch
    for k in range(warmup):
        x = xs[k]
        A.aica_bin(d, x)
        A.aica_forces(d, x, sp, wl.eps, wl.sigma, precision=precision)
        if adjoint:
            A.aica_forces_adjoint(d, x, G, GAMMA, sp, wl.eps, wl.sigma, precision=precision)
    torch.cuda.synchronize()
    for k in TIMERS:
        d.profile_read(k, reset=True)
    d.profile(True)
    torch.cuda.synchronize()
    counts, routes = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        x = xs[warmup + k]
        A.aica_bin(d, x)  # synchronises once (unlocated and reaction-slot counts): the route counts are host-side
        inf = d.info()
        routes.append((inf["located_ball"], inf["located_record"], inf["located_search"]))
        F, uw, npairs = A.aica_forces(d, x, sp, wl.eps, wl.sigma, precision=precision)
        counts.append(npairs)
        if adjoint:
            A.aica_forces_adjoint(d, x, G, GAMMA, sp, wl.eps, wl.sigma, precision=precision)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    d.profile(False)
    prof = {k: d.profile_read(k, reset=True) for k in TIMERS}
    return t, prof, [int(c.item()) for c in counts], routes


def evaluate(A, d, x, sp, wl, G, precision):
    """Forces, U/W, npairs and dL/dx on one position set (untimed; for the error statements)."""
    A.aica_bin(d, x)
    F, uw, npairs = A.aica_forces(d, x, sp, wl.eps, wl.sigma, precision=precision)
    gx, ge, gs = A.aica_forces_adjoint(d, x, G, GAMMA, sp, wl.eps, wl.sigma, precision=precision)
    return (F.double().cpu().numpy(), uw.cpu().numpy(), int(npairs.item()), gx.double().cpu().numpy(),
            ge.cpu().numpy(), gs.cpu().numpy())


def stored_binary_errors(wl, G, results):
    """Errors of the GPU adjoint against the stored FP64 oracle results of the binary mixture (dL/dx on
    1,024 fixed rows relative to the rms over all molecules; the four parameter gradients against the
    oracle's analytic values and against its central differences at h = 1e-6; L)."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_binary_adjoint as M
    g = M.read()
    assert wl.n == int(g["n"]) and GAMMA == wl.extra["gamma"]
    out = {}
    for prec, (F, uw, gx, ge, gs) in results.items():
        L = float((G * F).sum() + GAMMA * uw[0])
        out[f"stored_{prec}_dLdx_rows"] = float(np.abs(gx[g["rows"]] - g["dLdx"]).max() / g["rms_dLdx_all"])
        out[f"stored_{prec}_dparams"] = float(max((np.abs(ge - g["grad_eps"]) / np.abs(g["grad_eps"])).max(),
                                                  (np.abs(gs - g["grad_sigma"]) / np.abs(g["grad_sigma"])).max()))
        out[f"stored_{prec}_dparams_vs_fd"] = float(max((np.abs(ge - g["fd_eps"]) / np.abs(g["fd_eps"])).max(),
                                                        (np.abs(gs - g["fd_sigma"]) / np.abs(g["fd_sigma"])).max()))
        out[f"stored_{prec}_L"] = abs(L - g["L"]) / abs(g["L"])
    out["stored_rows"] = len(g["rows"])
    return out


def cpu_baseline(wl, seconds_target, F32, F64, G, gx32, gx64, rng_seed=7):
    """Time the FP64 oracle on a bounded sample of rows (each row against every molecule and image),
    extrapolate to all rows, and compare the GPU forces on the same rows; then compare the GPU adjoint's
    dL/dx with the oracle's on a third of those rows (not timed)."""
    from oracle import oracle as O
    O.lib()
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(rng_seed)
    n = wl.n
    # calibrate on a few rows, then size the sample for the time target
    r0 = rng.choice(n, min(n, 4 * cores), replace=False)
    t = time.perf_counter()
    O.forces_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, r0, rot=wl.rotations)
    per_row = (time.perf_counter() - t) / len(r0)
    nrows = int(min(n, max(len(r0), seconds_target / max(per_row, 1e-9))))
    rows = rng.choice(n, nrows, replace=False)
    t = time.perf_counter()
    Fr, Ur, Wr, cnt = O.forces_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, rows,
                                    rot=wl.rotations)
    t = time.perf_counter() - t
    t_full = t * n / nrows
    rms = np.sqrt((Fr ** 2).sum(1).mean())
    errs = {}
    for name, F in (("fp32", F32), ("fp64", F64)):
        if F is not None:
            errs[f"e_F_{name}"] = float(np.sqrt(((F[rows] - Fr) ** 2).sum(1)).max() / rms)
    errs["e_F_rows"] = nrows
    arows = rows[:max(1, nrows // 3)]
    rg = O.adjoint_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, GAMMA, arows,
                        rot=wl.rotations)
    grms = np.sqrt((rg ** 2).mean())
    for name, gx in (("fp32", gx32), ("fp64", gx64)):
        if gx is not None:
            errs[f"e_dLdx_{name}"] = float(np.abs(gx[arows] - rg).max() / grms)
    errs["e_dLdx_rows"] = len(arows)
    return {"seconds": t, "rows": nrows, "t_full": t_full, "cores": cores, "row_pairs": int(cnt.sum()),
            "errors": errs}


VALU_ISSUE_PEAK = 256 * 2.4e9  # one 64-lane VALU instruction per CU per cycle


def pmc_summary(paths, calib_fetch=None, calib_write=None, calib_mib=512):
    """Summarise rocprofv3 --pmc counter CSVs (run_counter_collection.csv): per kernel the dispatch count,
    mean duration under counters and the mean of every counter per dispatch; then, for the pair kernels,
    the lines the benchmark reads: VALU issue fraction (SQ_INSTS_VALU over the duration against one
    instruction per CU per cycle), executed FLOPs (64 lanes x the FLOPS_FP32/_FP64 counters and their
    transcendental parts, which count per wave instruction) and HBM traffic (FETCH_SIZE and WRITE_SIZE in
    KiB with the scale of the same counter on a device copy of known size)."""
    import csv
    import re
    def load(path):
        acc, dur = {}, {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k = re.sub(r"\(.*", "", r["Kernel_Name"].replace("void (anonymous namespace)::", "")
                           .replace("(anonymous namespace)::", ""))
                per = acc.setdefault(k, {}).setdefault(r["Counter_Name"], {})
                per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
                dur.setdefault(k, {})[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        return acc, dur
    acc, dur = {}, {}
    for p in paths:
        a, d = load(p)
        for k in a:
            for c, v in a[k].items():
                acc.setdefault(k, {})[c] = v
            dur.setdefault(k, {}).update({(p, i): t for i, t in d[k].items()})
    mean = {k: {c: sum(v.values()) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    scale = {}
    for name, path in (("FETCH_SIZE", calib_fetch), ("WRITE_SIZE", calib_write)):
        if path:
            a, _ = load(path)
            vals = [sum(v.values()) / len(v) for k, cs in a.items() if "copyBuffer" in k for c, v in cs.items()
                    if c == name]
            nbytes = float(calib_mib) * (1 << 20)
            scale[name] = nbytes / 1024 / vals[0] if vals else None
    names = sorted({c for cs in mean.values() for c in cs})
    short = [n.replace("SQ_INSTS_VALU_", "").replace("SQ_INSTS_", "").replace("SQ_", "") for n in names]
    lines = ["# counter columns: " + ", ".join(names),
             f"# {'kernel':40s} {'ms(pmc)':>8s} " + " ".join(f"{n[:11]:>11s}" for n in short)]
    for k in sorted(mean, key=lambda k: -sum(dur[k].values()) / len(dur[k])):
        ms = 1e3 * sum(dur[k].values()) / len(dur[k])
        if ms < 0.01:
            continue
        lines.append(f"# {k[:40]:40s} {ms:8.3f} " + " ".join(f"{mean[k].get(n, 0.0):11.4e}" for n in names))
    for key, kern in PAIR_KERNELS.items():
        if kern not in mean:
            continue
        m, t = mean[kern], sum(dur[kern].values()) / len(dur[kern])
        if "SQ_INSTS_VALU" in m:
            lines.append(f"issue: {key} {m['SQ_INSTS_VALU'] / t / VALU_ISSUE_PEAK:.4f}")
        fl = [c for c in ("SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_FLOPS_FP32_TRANS", "SQ_INSTS_VALU_FLOPS_FP64",
                          "SQ_INSTS_VALU_FLOPS_FP64_TRANS") if c in m]
        if len(fl) == 4:
            lines.append(f"flops: {key} {64 * sum(m[c] for c in fl):.6e}")
        if "FETCH_SIZE" in m and "WRITE_SIZE" in m and scale.get("FETCH_SIZE") and scale.get("WRITE_SIZE"):
            lines.append(f"traffic: {key} {m['FETCH_SIZE']:.1f} {scale['FETCH_SIZE']:.4f} {m['WRITE_SIZE']:.1f} "
                         f"{scale['WRITE_SIZE']:.4f}")
    lines.append(f"sources_sha256: {kernel_digest()}")
    return "\n".join(lines)


def trace_summary(path):
    """Summarise a rocprofv3 --kernel-trace --stats run_kernel_stats.csv: per kernel the calls and the mean,
    smallest and largest duration (microseconds) and the share of the total kernel time."""
    import csv
    import re
    lines = [f"# {'kernel':46s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    with open(path) as fh:
        for r in csv.DictReader(fh):
            k = re.sub(r"\(.*", "", r["Name"].replace("void (anonymous namespace)::", "")
                       .replace("(anonymous namespace)::", ""))
            if float(r["Percentage"]) < 0.05:
                continue
            lines.append(f"  {k[:46]:46s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
                         f"{float(r['MinNs']) / 1e3:10.1f} {float(r['MaxNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}")
    lines.append(f"# kernel sources sha256 (first 16 hex): {kernel_digest()}")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates the FETCH_SIZE and "
                         "WRITE_SIZE counters against a kernel of known traffic) and exit")
    ap.add_argument("--pmc-summary", nargs="+", metavar="CSV",
                    help="only summarise rocprofv3 --pmc output (run_counter_collection.csv files) and exit")
    ap.add_argument("--calib-fetch", metavar="CSV", help="with --pmc-summary: FETCH_SIZE run of --copy-calibration")
    ap.add_argument("--calib-write", metavar="CSV", help="with --pmc-summary: WRITE_SIZE run of --copy-calibration")
    ap.add_argument("--calib-mib", type=int, default=512, help="with --pmc-summary: MiB of the calibration copy")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="only summarise a rocprofv3 --kernel-trace --stats run_kernel_stats.csv and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary, args.calib_fetch, args.calib_write, args.calib_mib))
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; multi-GPU runs (processor referral "
                                   "and halo exchange) are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_cs_0702131_amd as A
    from paper_cs_0702131_amd import workloads as W

    t0 = time.perf_counter()
    wl = workload(args.workload)
    log(f"workload {wl.name}: {wl.mesh.n_cells} cells, {wl.n} molecules ({time.perf_counter() - t0:.1f}s)")
    t0 = time.perf_counter()
    d = A.DIL(wl.mesh, wl.rcut)
    info = d.info()
    log(f"interaction lists: {info['n_dil']} cell pairs in {info['build_seconds']:.1f}s")

    dev = torch.device("cuda:0")
    S = args.warmup + args.steps
    t0 = time.perf_counter()
    sets = moving_sets(wl, S)
    xs32 = [torch.tensor(x, dtype=torch.float32, device=dev) for x in sets]
    xs64 = None if args.no_fp64 else [torch.tensor(x, dtype=torch.float64, device=dev) for x in sets]
    del sets
    log(f"{S} moving position sets resident in HBM ({time.perf_counter() - t0:.1f}s)")
    sp = torch.tensor(wl.species, dtype=torch.int32, device=dev)
    G = wl.extra.get("G")
    if G is None:
        G = W.qround(np.random.default_rng(9).standard_normal((wl.n, 3)))
    G32 = torch.tensor(G, dtype=torch.float32, device=dev)
    G64 = torch.tensor(G, dtype=torch.float64, device=dev)

    res = {}
    t, prof, counts, routes = timed_steps(A, d, xs32, sp, wl, G32, "fp32", args.steps, args.warmup)
    res["fp32_fwd_adj"] = (t, prof, counts)
    log(f"fp32 fwd+adj: {1e3 * t / args.steps:.3f} ms/step, npairs {counts}")
    t, prof, c, _ = timed_steps(A, d, xs32, sp, wl, G32, "fp32", args.steps, args.warmup, adjoint=False)
    res["fp32_fwd"] = (t, prof, c)
    assert c == counts
    if xs64 is not None:
        t, prof, c, _ = timed_steps(A, d, xs64, sp, wl, G64, "fp64", args.steps, args.warmup)
        res["fp64_fwd_adj"] = (t, prof, c)
        assert c == counts, (c, counts)
        t, prof, c, _ = timed_steps(A, d, xs64, sp, wl, G64, "fp64", args.steps, args.warmup, adjoint=False)
        res["fp64_fwd"] = (t, prof, c)
        log(f"fp64 fwd+adj: {1e3 * res['fp64_fwd_adj'][0] / args.steps:.3f} ms/step")

    # error statements and work counts on the first position set (untimed)
    F32n, uw32, npairs, gx32n, ge32, gs32 = evaluate(A, d, xs32[0], sp, wl, G32, "fp32")
    info = d.info()
    dil_cand, lane_pairs = d.work_stats()
    log(f"groups {info['n_groups']} group pairs {info['n_group_pairs']} ({info['group_seconds']:.1f}s); "
        f"DIL candidates {dil_cand}, executed lane pairs {lane_pairs}")
    F64n = gx64n = None
    if xs64 is not None:
        F64n, uw64, npairs64, gx64n, ge64, gs64 = evaluate(A, d, xs64[0], sp, wl, G64, "fp64")
        assert npairs64 == npairs, (npairs64, npairs)

    K = args.steps
    t_main, prof_main, counts_main = res["fp32_fwd_adj"]
    value = sum(counts_main) / t_main
    breakdown = {}
    for key, (t, prof, c) in res.items():
        breakdown[key] = {"ms_per_step": 1e3 * t / K, "pairs_per_s": sum(c) / t,
                          **{f"{k}_ms": v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}}
    # dominant kernel of the FP32 step and its algorithmic FLOP rate (work counts of the first set)
    fwd_ms = prof_main["pair_fwd"][0] / prof_main["pair_fwd"][1]
    adj_ms = prof_main["pair_adj"][0] / prof_main["pair_adj"][1]
    rejected = dil_cand - npairs
    if adj_ms >= fwd_ms:
        kname, kms, flops = "pair_adj", adj_ms, FLOP_ADJ_PAIR * npairs + FLOP_REJECT * rejected
    else:
        kname, kms, flops = "pair_fwd", fwd_ms, FLOP_FWD_PAIR * npairs + FLOP_REJECT * rejected
    achieved = flops / (kms * 1e-3) / 1e12
    ctr = measured_counters(kname, args.workload)
    ex = ctr.get("executed_flop")
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": ctr.get("traffic"), "traffic_unit": "bytes per launch",
                "valu_issue_frac": ctr.get("valu_issue_frac"),
                "executed_tflops": None if ex is None else ex / (kms * 1e-3) / 1e12,
                "executed_frac": None if ex is None else ex / (kms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                "kernel": kname,
                "kernel_ms": kms, "algorithmic_flop": flops}

    cpu = None
    errors = {"npairs": npairs}
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, args.cpu_seconds, F32n, F64n, G, gx32n, gx64n)
        cpu = {"value": npairs / cb["t_full"], "unit": "pair interactions/s", "cores": cb["cores"],
               "kind": "oracle",
               "sample": f"{cb['rows']} random rows of {wl.n} (each against all molecules and images, "
                         f"{cb['seconds']:.1f}s), extrapolated linearly to all rows"}
        errors.update(cb["errors"])
    if F64n is not None:
        errors["e_F_fp32_vs_fp64_gpu"] = float(np.sqrt(((F32n - F64n) ** 2).sum(1)).max()
                                               / np.sqrt((F64n ** 2).sum(1).mean()))
        errors["dU_fp32_vs_fp64"] = float(abs(uw32[0].item() - uw64[0].item()) / abs(uw64[0].item()))
        errors["dW_fp32_vs_fp64"] = float(abs(uw32[1].item() - uw64[1].item()) / abs(uw64[1].item()))
        # every row of dL/dx (the FP64 path matches the oracle to ~1e-15 on the sampled rows)
        errors["e_dLdx_fp32_vs_fp64_gpu"] = float(np.abs(gx32n - gx64n).max() / np.sqrt((gx64n ** 2).mean()))
    if args.workload == "binary":
        res_b = {"fp32": (F32n, uw32, gx32n, ge32, gs32)}
        if F64n is not None:
            res_b["fp64"] = (F64n, uw64, gx64n, ge64, gs64)
        errors.update(stored_binary_errors(wl, G, res_b))

    out = {"metric": METRIC, "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_main / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": wl.name, "cells": wl.mesh.n_cells, "molecules": wl.n, "npairs": npairs,
                      "npairs_per_step": counts_main, "located_ball_record_search": routes,
                      "step": "aica_bin + aica_forces + aica_forces_adjoint on moving molecules",
                      "parallelism": "single GPU",
                      "dil_cell_pairs": info["n_dil"], "dil_candidates": dil_cand, "lane_pairs": lane_pairs,
                      "lane_efficiency": npairs / max(lane_pairs, 1)},
           "breakdown": breakdown, "errors": errors, "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
