#!/usr/bin/env python3
"""Benchmark of the HTLR matrix-vector product on one MI355X.

A step is one HTLR product f = A u (near field + diagonal, up contraction,
core apply and down expansion on every level) on a matrix already built and
resident in HBM, with u resident in HBM.  Prints one compact JSON line on
stdout; the full record of every block goes to stderr as a line starting
with "[bench-detail]".

Headline workload: d = 3, n = 128 (N = 2,097,152), k = 1/|x-y|, p = 8,
leaf 8^3, a = 1, 16 right-hand sides u ~ N(0,1) (seed 2), FP64.  The same
products in FP32 and bfloat16-core precision are sub-results with their
errors against the FP64 product.  Further blocks: the n = 64 FP64 product,
construction at the paper's table shapes, the QR / QRCP forms, the
quasi-uniform transfer form, the warped-grid solve and the request server.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HTLR matvec Gpt/s + solves/s at stated err vs FP64; p50/p99 solve latency"
PEAK = {  # MI355X published peaks (dense), TFLOP/s
    "fp64_vector": 78.6, "fp32_vector": 157.3, "fp64_mfma": 78.6, "fp32_mfma": 157.3, "bf16_mfma": 2500.0,
}
HBM_GBS = 8000.0
KERNEL_LABEL = {"inv_r": "1/|x-y|", "neg_log": "-log|x-y|", "exp": "exp(-|x-y|)", "gauss": "exp(-|x-y|^2/(2d))"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="w3d_invr_n128_r16")
    ap.add_argument("--prec", default="fp64", help="fp64 | fp32 | bf16")
    ap.add_argument("--prof-steps", type=int, default=3,
                    help="steps of the profiled pass that times each kernel for the roofline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32 / bfloat16-core variants of the headline")
    ap.add_argument("--no-small", action="store_true", help="skip the n = 64 FP64 block")
    ap.add_argument("--cpu-leaves", type=int, default=64, help="leaf boxes of the CPU-oracle sample")
    ap.add_argument("--cpu-procs", type=int, default=16, help="worker processes of the CPU-oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the warped-grid solve block")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving block")
    ap.add_argument("--no-quasi", action="store_true", help="skip the quasi-uniform transfer block")
    ap.add_argument("--no-orth", action="store_true", help="skip the orthonormal / QRCP forms block")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-rates", default="0.25,0.5,1,2,4",
                    help="Poisson arrival rates as multiples of the measured capacity, comma separated")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the headline product (otherwise its built-in kernel choices, the ones the "
                         "full-size parity tests cover)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2508_05958_amd", "tuned_mi355x.txt"),
                    help="autotuner cache file (HTLR_TUNE_CACHE) used by the n = 64 block unless that variable is "
                         "set; its lines are the tuner's own output, so runs of the same shape use the same kernel "
                         "variants")
    ap.add_argument("--no-tables", action="store_true", help="skip construction at the paper's table shapes")
    ap.add_argument("--serial", action="store_true",
                    help="time the profiled, serially issued product (for kernel-trace runs: every kernel's "
                         "duration is its own, as in the roofline pass)")
    ap.add_argument("--write-traffic", action="store_true",
                    help="with --summarize-profile: store per-launch HBM bytes for the roofline's traffic field")
    ap.add_argument("--summarize-counters", default=None, metavar="DIR",
                    help="print a markdown summary of rocprofv3 SQ counter passes (p1/, p2/) and exit")
    ap.add_argument("--summarize-profile", default=None, metavar="DIR",
                    help="print a markdown summary of a rocprofv3 run directory (stats/, fetch/, write/) and exit")
    ap.add_argument("--profile-command", default="", help="command line recorded in the summary")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-out", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-pick", default=None, help=argparse.SUPPRESS)
    return ap.parse_args()


def level_shapes(info, w):
    """(level, boxes per dimension B, box side m) of every level."""
    return [(l, 2 ** l, w.n // 2 ** l) for l in range(info["levels"] + 1)]


# Kernel evaluations per second a tensor-grid product can reach when it is
# bound by the vector ALU (cores and near-field blocks made in the product).
# One evaluation of a radial kernel, per lane: 4 full-rate instructions
# (difference, r^2, scale, accumulate; 16 lanes per SIMD and cycle) and 2
# transcendentals (square root or reciprocal square root, and 2^x or log2; a
# quarter of that rate), i.e. 4/16 + 2/4 = 0.75 SIMD cycles.  1024 SIMDs at
# 2.4 GHz.  In FP64 the exp and log are software sequences; the same count
# is used as a lower bound on their cost.
EVAL_CYCLES = 0.75
EVAL_PEAK_G = 1024 * 2.4e9 / EVAL_CYCLES / 1e9


def algorithmic_cost(info, w, nrhs, prec):
    """Per launch of each product step: algorithmic flops (no padding),
    algorithmic HBM bytes (each operand read once, each result written
    once), and, on tensor grids, the kernel evaluations the step makes."""
    M = info["leaf_side"] ** w.d
    ev = 8 if prec == "fp64" else 4                      # vector and work-buffer element
    eg = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]         # core and staged source-tensor element
    N = w.N
    tensor = w.grid != "uniform"
    cost = {"near": (2.0 * info["near_pairs"] * M * M * nrhs, 2.0 * N * nrhs * ev,
                     float(info["near_pairs"] * M * M) if tensor else 0.0)}
    for l, B, m in level_shapes(info, w):
        pairs = info["adm_pairs"][l]
        if not pairs:
            continue
        r = info["level_rank"][l] or w.p                 # the level's Tucker rank (p unless truncated)
        P = r ** w.d
        nbox = B ** w.d
        wbytes = nbox * P * nrhs
        cost[f"up_l{l}"] = (2.0 * nbox * nrhs * sum(m ** (w.d - k) * r ** (k + 1) for k in range(w.d)),
                            N * nrhs * ev + wbytes * eg, 0.0)
        cost[f"core_l{l}"] = (2.0 * pairs * P * P * nrhs,
                              info["unique_cores"][l] * P * P * eg + wbytes * eg + wbytes * ev,
                              float(pairs * P * P) if tensor else 0.0)
        cost[f"down_l{l}"] = (2.0 * nbox * nrhs * sum(r ** (w.d - k) * m ** (k + 1) for k in range(w.d)),
                              wbytes * ev + 2.0 * N * nrhs * ev, 0.0)
    return cost


def peak_for(step, prec):
    """(bound, peak TFLOP/s) of a step.  The near field of these workloads
    (uniform 3D grid, 8^3-point leaves, radial kernel) runs on the matrix
    cores in FP64, or FP32 for the FP32 and bfloat16-core products; the up
    and down contractions are bound by HBM."""
    if step.startswith("up") or step.startswith("down"):
        return ("hbm", None)
    if step == "near":
        return ("mfma", PEAK["fp64_mfma"] if prec == "fp64" else PEAK["fp32_mfma"])
    return ("mfma", {"fp64": PEAK["fp64_mfma"], "fp32": PEAK["fp32_mfma"], "bf16": PEAK["bf16_mfma"]}[prec])


# Sources that define the product's kernels and work lists: a committed
# counter summary is used only while these are unchanged (the solver, server,
# transfer-form and no-allocation sources do not change a product's kernels).
PRODUCT_SOURCES = ("htlr_build.hip", "htlr_core_mfma.hip", "htlr_device.h", "htlr_handle.h", "htlr_internal.h",
                   "htlr_matvec.hip", "htlr_near_leaves.hip", "htlr_near_rows.hip", "htlr_plan.cpp")


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2508_05958_amd", "csrc")
    for name in PRODUCT_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload, prec, step, launches):
    """HBM bytes per launch from committed counter summaries, if they were
    taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    # counters are kept per kernel family: the near-field kernel, and the core
    # apply's largest dispatch (the deepest level, which dominates)
    key = "near" if step == "near" else ("core" if step.startswith("core") else step)
    if t.get("source_digest") != source_digest() or key not in t.get("kernels", {}):
        return None
    return t["kernels"][key]["hbm_bytes_per_launch"]


def to_device(torch, u, dt):
    """Column-major device copy of u ((N,) or (N, nrhs))."""
    if u.ndim == 2:
        return torch.tensor(u.T.copy(), dtype=dt, device="cuda").t()
    return torch.tensor(u, dtype=dt, device="cuda")


def np_mod():
    import numpy
    return numpy


def build_workload(H, np, w):
    """The workload's matrix: the uniform grid, or a warped tensor grid from
    its nodes (cores and near-field blocks then made in the product)."""
    if w.grid == "uniform":
        return H.htlr_build(None, w.kernel, w.d, w.n, w.p, w.leaf, a=w.a())
    return H.htlr_build(np.concatenate(w.nodes()), w.kernel, w.d, w.n, w.p, w.leaf, a=w.a(),
                        precisions=["fp64", "fp32"])


def run_workload(H, torch, w, prec, steps, warmup, prof_steps=3, tune=False, serial=False, M=None, ut=None):
    build_s = 0.0
    if M is None:
        t0 = time.time()
        M = build_workload(H, np_mod(), w)
        torch.cuda.synchronize()
        build_s = time.time() - t0
    info = M.info()
    if ut is None:
        ut = to_device(torch, w.rhs(), torch.float64 if prec == "fp64" else torch.float32)
    nrhs = 1 if ut.dim() == 1 else ut.shape[1]
    if tune:
        # kernel variants chosen by timing (the server does this per structure);
        # outside the timed region, like the build
        M.autotune(nrhs, prec)
    if serial:
        M.profile(True)          # every product of this run issued in order, warm-up included
    f = M.matvec(ut, prec=prec)
    for _ in range(warmup):
        M.matvec(ut, f, prec=prec)
    torch.cuda.synchronize()
    # timed region: the product as it runs in use (levels concurrent), or
    # with serial=True the profiled, serially issued product
    if serial:
        M.profile(True)          # clears the record
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        M.matvec(ut, f, prec=prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / steps * 1e3
    if not serial:
        # per-kernel durations: a second pass with the profiler on, which
        # issues every launch in order so that each duration is the kernel's own
        M.profile(True)
        torch.cuda.synchronize()
        for _ in range(max(1, prof_steps)):
            M.matvec(ut, f, prec=prec)
        torch.cuda.synchronize()
    prof = M.profile_read()
    M.profile(False)
    return M, info, f, nrhs, ms, prof, build_s


def roofline(info, w, prec, nrhs, prof, ms_meas, workload):
    """The dominant kernel against its roofline, every kernel's own fraction,
    and the whole product's T_roof / T_meas, T_roof = sum over steps of
    max(algorithmic bytes / HBM bandwidth, algorithmic flops / peak)."""
    cost = algorithmic_cost(info, w, nrhs, prec)
    per = {}
    t_roof = 0.0
    for step, (launches, total) in prof.items():
        avg = total / max(launches, 1)
        if step not in cost:
            per[step] = {"ms": round(avg, 4)}
            continue
        flops, nbytes, evals = cost[step]
        bound, peak = peak_for(step, prec)
        t_mem = nbytes / (HBM_GBS * 1e9) * 1e3
        if evals > 0:
            # tensor grid: cores and near-field blocks evaluated in the product
            rate = evals / (avg * 1e-3) / 1e9
            per[step] = {"ms": round(avg, 4), "bound": "alu", "achieved_Geval_s": round(rate, 1),
                         "peak_Geval_s": round(EVAL_PEAK_G, 1), "frac": round(rate / EVAL_PEAK_G, 4)}
            t_roof += max(t_mem, evals / (EVAL_PEAK_G * 1e9) * 1e3)
        elif bound == "hbm":
            gbs = nbytes / (avg * 1e-3) / 1e9
            per[step] = {"ms": round(avg, 4), "bound": "hbm", "achieved_GBs": round(gbs, 1),
                         "frac": round(gbs / HBM_GBS, 4)}
            t_roof += t_mem
        else:
            ach = flops / (avg * 1e-3) / 1e12
            per[step] = {"ms": round(avg, 4), "bound": bound, "achieved_tflops": round(ach, 2), "peak_tflops": peak,
                         "frac": round(ach / peak, 4)}
            t_roof += max(t_mem, flops / (peak * 1e12) * 1e3)
    mf = [s for s in per if s in cost and per[s]["bound"] != "hbm"]
    dom = max(mf, key=lambda s: per[s]["ms"])
    d = per[dom]
    if d["bound"] == "alu":
        roof = {"bound": "alu", "achieved": d["achieved_Geval_s"], "peak": d["peak_Geval_s"], "unit": "Geval/s",
                "frac": d["frac"], "traffic": traffic_for(workload, prec, dom, prof[dom][0]), "kernel": dom,
                "evals_per_launch": cost[dom][2], "avg_launch_ms": d["ms"],
                "product_frac": round(t_roof / ms_meas, 4), "T_roof_ms": round(t_roof, 3)}
    else:
        roof = {"bound": d["bound"], "achieved": d["achieved_tflops"], "peak": d["peak_tflops"], "unit": "TFLOP/s",
                "frac": d["frac"], "traffic": traffic_for(workload, prec, dom, prof[dom][0]),
                "kernel": dom, "flop_per_launch": cost[dom][0], "avg_launch_ms": d["ms"],
                "product_frac": round(t_roof / ms_meas, 4), "T_roof_ms": round(t_roof, 3)}
    return roof, per


def cpu_worker(wname, leaves_csv, out):
    """One process of the CPU baseline: builds the oracle's tree and inputs
    (not timed), reports ready, waits for "go" on stdin, then computes the
    oracle rows of its leaf boxes and saves them to ``out``."""
    import numpy as np
    import htlr_workloads as W
    from oracle import geometry, htlr
    w = W.WORKLOADS[wname]
    g = geometry.uniform_grid(w.d, w.n) if w.grid == "uniform" else geometry.tensor_grid(w.nodes())
    O = htlr.HTLR(g, w.kernel, w.p, w.leaf, w.a())
    u = w.rhs() if w.grid == "uniform" else W.solve_target(w.points())
    leaves = O.tree.leaves()
    pick = [leaves[int(i)] for i in leaves_csv.split(",")]
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.perf_counter()
    vals = [O.matvec(u, [nd]) for nd in pick]
    busy = time.perf_counter() - t0
    np.savez(out, rows=O.leaf_rows(pick), vals=np.concatenate([v.reshape(v.shape[0], -1) for v in vals]),
             busy=busy)
    print("done", flush=True)


def host_cpu():
    model = ""
    try:
        import subprocess
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return os.cpu_count(), model


def cpu_baseline(w, count, procs, f_gpu):
    """The CPU FP64 HTLR oracle on a seeded sample of leaf boxes of the
    workload, spread over worker processes (one BLAS thread each), timed from
    the moment every worker is initialised; also returns the relative error
    of the GPU rows against the oracle's.  Each worker is a child process
    that is waited for, so none outlives the benchmark."""
    import shutil
    import subprocess
    import tempfile

    import numpy as np
    import htlr_workloads as W
    side = w.n
    while side > w.leaf:
        side //= 2
    nleaves = (w.n // side) ** w.d
    pick = [int(i) for i in W.sample_leaves(w.seed, nleaves, count)]
    procs = max(1, min(procs, len(pick), os.cpu_count() or 1))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    tmp = tempfile.mkdtemp(prefix="htlr_cpu_")
    workers = []
    try:
        for k in range(procs):
            mine = pick[k::procs]
            out = os.path.join(tmp, f"w{k}.npz")
            p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", w.name,
                                  "--cpu-out", out, "--cpu-pick", ",".join(map(str, mine))],
                                 stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env, cwd=ROOT)
            workers.append((p, out))
        for p, _ in workers:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("CPU baseline worker failed to start")
        t0 = time.perf_counter()
        for p, _ in workers:
            p.stdin.write("go\n")
            p.stdin.flush()
        for p, _ in workers:
            p.stdout.readline()
            p.wait()
        wall = time.perf_counter() - t0
        res = [np.load(out) for _, out in workers]
    finally:
        for p, _ in workers:
            if p.poll() is None:
                p.kill()
                p.wait()
        shutil.rmtree(tmp, ignore_errors=True)
    rows = np.concatenate([r["rows"] for r in res])
    vals = np.concatenate([r["vals"] for r in res])
    busy = float(sum(r["busy"] for r in res))
    npts = len(rows) * w.nrhs
    fg = f_gpu.reshape(w.N, -1)[rows]
    err = float(np.linalg.norm(fg - vals) / np.linalg.norm(vals))
    ncpu, model = host_cpu()
    return {"value": npts / wall / 1e9, "unit": "Gpt/s", "cores": procs, "kind": "oracle",
            "sample": f"{len(pick)} seeded leaf boxes of {nleaves} ({len(rows)} rows x {w.nrhs} rhs) of {w.name}: "
                      f"plain NumPy FP64 HTLR product (Alg. 4.2) restricted to those rows, scaled by the rows "
                      f"computed; {procs} processes x 1 BLAS thread, {wall:.1f} s wall, {busy:.1f} s CPU",
            "host_cpus": ncpu, "host_model": model}, err


# Construction at the shapes of the paper's Tables 5.1-5.4 (a = 0, FP64):
# (table, d, kernel, admissibility, p, leaf threshold, n, the paper's
# printed t_c in s, m_h in GB on its CPU and e_apply;rand).  Strong admissibility takes
# eta^2 = d, as in Prop. 3.9; the paper's kernels carry constants 1/(2 pi),
# 1/(4 pi) that do not change relative errors or timings.
PAPER_SHAPES = [
    ("5.1", 2, "gauss", "weak", 8, 16, [(256, 1.5, 0.16, 1.3e-11), (512, 3.8, 0.65, 2.1e-11), (1024, 16, 2.6, 1.5e-10),
                                        (2048, 68, 10, 2.0e-11), (4096, 280, 41, 1.8e-11)]),
    ("5.2", 2, "neg_log", "strong", 8, 16, [(256, 7.6, 1.3, 1.1e-7), (512, 30, 5.4, 8.1e-8), (1024, 130, 23, 1.2e-7),
                                            (2048, 540, 92, 5.3e-8), (4096, 2100, 370, 4.4e-8)]),
    ("5.3", 3, "gauss", "weak", 4, 5, [(32, 4.0, 0.14, 2.3e-5), (64, 27, 1.2, 7.4e-6), (128, 220, 9.2, 8.6e-6),
                                       (256, 1800, 74, 1.2e-5)]),
    ("5.4", 3, "inv_r", "strong", 4, 5, [(32, 48, 2.1, 1.9e-4), (64, 540, 23, 2.6e-4), (128, 5100, 210, 3.1e-4)]),
]


def dense_row_errors(M, torch, w, u64, fs, size=1000):
    """e_apply;rand as Sec. 5 defines it, for each product in fs: the relative
    2-norm error against the uncompressed Nystrom product (eq. 1.3-1.4) on
    `size` seeded rows (all right-hand sides), those rows formed on the GPU
    by htlr_exact_rows in FP64."""
    pick = torch.tensor(w.rows(min(size, w.N)), device="cuda")
    if u64.dim() == 1:
        ex = M.exact_rows(u64, pick)
    else:
        ex = torch.cat([M.exact_rows(u64[:, c:c + 8], pick) for c in range(0, u64.shape[1], 8)], dim=1)
    nex = torch.linalg.norm(ex)
    return {k: float(f"{float(torch.linalg.norm(f.double()[pick] - ex) / nex):.3g}") for k, f in fs.items()}


def paper_tables_block(H, torch, np):
    """Build time t_c (host planning + GPU construction, synchronised), device
    bytes m_h and the FP64 product time at the paper's shapes.  Accuracy at
    these shapes is checked against the oracle in the GPU tests."""
    H.htlr_build(None, "gauss", 2, 64, 8, 16, a=np.zeros(64 * 64), admissibility="weak").free()   # warm-up
    rows = []
    for table, d, kern, adm, p, leaf, sizes in PAPER_SHAPES:
        for n, tc_paper, mh_paper, e_paper in sizes:
            N = n ** d
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = H.htlr_build(None, kern, d, n, p, leaf, a=np.zeros(N), eta2=float(d) if adm == "strong" else 1.0,
                             admissibility=adm, precisions=["fp64"])
            torch.cuda.synchronize()
            tc = time.perf_counter() - t0
            info = M.info()
            # e_apply;rand (Sec. 5): relative 2-norm error of the product
            # against the exact A u on 1000 random rows, u ~ N(0, 1)
            u = torch.tensor(np.random.default_rng([d, n]).standard_normal(N), device="cuda")
            pick = torch.tensor(np.sort(np.random.default_rng([d, n, 1]).choice(N, size=min(1000, N), replace=False)),
                                device="cuda")
            f = M.matvec(u, prec="fp64")
            ex = M.exact_rows(u, pick)
            e_apply = float(torch.linalg.norm(f[pick] - ex) / torch.linalg.norm(ex))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                M.matvec(u, f, prec="fp64")
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            rows.append({"table": table, "d": d, "kernel": KERNEL_LABEL[kern], "admissibility": adm, "p": p,
                         "leaf": leaf, "n": n, "N": N, "t_c_s": round(tc, 4),
                         "m_h_GB": round(info["device_bytes"] / 1e9, 4), "matvec_ms": round(ms, 3),
                         "e_apply_rand": float(f"{e_apply:.3g}"),
                         "paper_t_c_s": tc_paper, "paper_m_h_GB": mh_paper, "paper_e_apply_rand": e_paper})
            print(f"[bench]   table {table} n={n}: t_c {tc:.3f} s, {info['device_bytes'] / 1e9:.3f} GB, "
                  f"matvec {ms:.2f} ms, e_apply;rand {e_apply:.2e} (paper {e_paper:g})", file=sys.stderr, flush=True)
            M.free()
            del u, f
            torch.cuda.empty_cache()
    return {"note": "t_c and m_h as the paper's Tables 5.1-5.4 define them, on one MI355X; the paper's figures "
                    "are from a Xeon Gold 6226R in MATLAB and store one block per admissible leaf",
            "rows": rows}


def solve_block(H, torch, np, W):
    """Warped-grid solve A u = f, f = A u*: GMRES with FP32 inner products and
    FP64 refinement against plain FP64 GMRES, both to the same FP64 residual."""
    w = W.WORKLOADS["w3d_exp_warp_n96"]
    x = W.warped_nodes(w.n)
    pts = W.grid_points([x] * 3)
    a = 2.0 + pts[:, 0]
    t0 = time.time()
    M = H.htlr_build(np.concatenate([x] * 3), w.kernel, 3, w.n, w.p, w.leaf, a=a, precisions=["fp64", "fp32"])
    torch.cuda.synchronize()
    build_s = time.time() - t0
    us = torch.tensor(W.solve_target(pts), device="cuda")
    f = M.matvec(us, prec="fp64")
    out = {"workload": w.name, "N": w.N, "tol": 1e-10, "build_s": round(build_s, 3), "products": {}}
    # the products the solve is made of, per kernel against the evaluation-rate bound
    info = M.info()
    for pr in ("fp32", "fp64"):
        ut = us if pr == "fp64" else us.float()
        fp = M.matvec(ut, prec=pr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            M.matvec(ut, fp, prec=pr)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 3 * 1e3
        M.profile(True)
        M.matvec(ut, fp, prec=pr)
        torch.cuda.synchronize()
        prof = M.profile_read()
        M.profile(False)
        roof, per = roofline(info, w, pr, 1, prof, ms, w.name)
        out["products"][pr] = {"ms": round(ms, 3), "err_vs_fp64": float(torch.linalg.norm(fp.double() - f) /
                                                                       torch.linalg.norm(f)),
                               "roofline": roof, "kernels": per}
        print(f"[bench]   warped {pr} product {ms:.2f} ms: {roof['kernel']} {roof['achieved']} of {roof['peak']} "
              f"{roof['unit']} ({roof['frac']:.2f}), product {roof['product_frac']:.2f} of T_roof", file=sys.stderr,
              flush=True)
        del fp
    for inner in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info, st = M.solve(f, tol=1e-10, restart=30, inner_prec=inner, max_inner=600)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"inner_{inner}"] = {
            "seconds": round(dt, 3), "solves_per_s": round(1.0 / dt, 4), "points_per_s": round(w.N / dt, 1),
            "rel_residual_fp64": info.rel_residual, "outer_iters": info.outer_iters,
            "inner_iters": info.inner_iters, "matvecs_fp64": info.matvecs_fp64, "matvecs_inner": info.matvecs_inner,
            "rel_err_vs_ustar": float(torch.linalg.norm(u - us) / torch.linalg.norm(us)), "status": st}
    M.free()
    return out


def quasi_block(H, torch, np, W, steps=10):
    """Quasi-uniform grid through the uniform grid of m = 2n cells (the
    transfer form T Ahat S): product rate in FP64 and FP32, and the transfer
    kernels against HBM bandwidth.  Per launch the S transfer reads u (N
    values) and writes S u (M values); the T transfer reads Ahat S u (M),
    u and a (N each) and writes f (N)."""
    w = W.WORKLOADS["wq2d_log_n512_m1024"]
    nd = w.nodes()
    M_ = w.m ** w.d
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = H.htlr_build_quasi(np.concatenate(nd), w.kernel, w.d, w.n, w.m, w.p, w.leaf, a=w.a(), eta2=w.eta2,
                           precisions=["fp64", "fp32"])
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = A.info()
    out = {"workload": w.name, "d": w.d, "n": w.n, "N": w.N, "m": w.m, "M": M_, "rho": w.m / w.n,
           "kernel": KERNEL_LABEL.get(w.kernel, w.kernel), "p": w.p, "leaf": w.leaf,
           "admissibility": f"strong, eta^2={w.eta2:g}", "build_s": round(build_s, 3),
           "device_bytes": info["device_bytes"], "u": "smooth u(x) of the paper's quasi-uniform experiment"}
    u64 = torch.tensor(w.rhs(), dtype=torch.float64, device="cuda")
    for prec in ("fp64", "fp32"):
        u = u64 if prec == "fp64" else u64.float()
        f = A.matvec(u, prec=prec)
        for _ in range(2):
            A.matvec(u, f, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            A.matvec(u, f, prec=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        A.profile(True)
        for _ in range(steps):
            A.matvec(u, f, prec=prec)
        prof = A.profile_read()
        A.profile(False)
        esz = 8 if prec == "fp64" else 4
        kern = {}
        for name, nbytes in (("quasi_s", esz * (w.N + M_)), ("quasi_t", esz * (M_ + 3 * w.N))):
            launches, total = prof[name]
            avg = total / launches
            gbs = nbytes / (avg * 1e-3) / 1e9
            kern[name] = {"avg_launch_ms": round(avg, 4), "bound": "hbm", "algorithmic_bytes": nbytes,
                          "achieved_GBs": round(gbs, 1), "peak_GBs": HBM_GBS,
                          "frac": round(gbs / HBM_GBS, 4)}
        inner_ms = sum(t for k, (c, t) in prof.items() if not k.startswith("quasi")) / steps
        out[prec] = {"ms_per_product": round(ms, 4), "Gpt_s": round(w.N / (ms * 1e-3) / 1e9, 5),
                     "ahat_ms_profiled": round(inner_ms, 4), "transfers": kern,
                     "transfer_share": round(sum(v["avg_launch_ms"] for v in kern.values())
                                             / (inner_ms + sum(v["avg_launch_ms"] for v in kern.values())), 4)}
        print(f"[bench]   quasi {prec}: {ms:.3f} ms/product, S {kern['quasi_s']['avg_launch_ms']:.4f} ms "
              f"({kern['quasi_s']['frac']:.2f} of HBM), T {kern['quasi_t']['avg_launch_ms']:.4f} ms",
              file=sys.stderr, flush=True)
        del f
    A.free()
    # oversampling sweep (the paper's quasi-uniform experiment varies rho):
    # the transfer form at m = rho n against the direct HTLR product on the
    # same warped tensor grid (Def. 3.5, cores made in the product), which
    # approximates the Nystrom operator at the warped points to the HTLR
    # accuracy; FP64, u = the smooth u above
    D = H.htlr_build(np.concatenate(nd), w.kernel, w.d, w.n, w.p, w.leaf, a=w.a(), eta2=w.eta2, precisions=["fp64"])
    fd = D.matvec(u64, prec="fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        D.matvec(u64, fd, prec="fp64")
    torch.cuda.synchronize()
    out["direct_tensor_grid_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 4)
    D.free()
    sweep = []
    for m in (w.n, 2 * w.n, 4 * w.n):
        Q = H.htlr_build_quasi(np.concatenate(nd), w.kernel, w.d, w.n, m, w.p, w.leaf, a=w.a(), eta2=w.eta2,
                               precisions=["fp64"])
        fq = Q.matvec(u64, prec="fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            Q.matvec(u64, fq, prec="fp64")
        torch.cuda.synchronize()
        sweep.append({"m": m, "rho": m / w.n, "ms_per_product": round((time.perf_counter() - t0) / 5 * 1e3, 4),
                      "rel_diff_vs_direct": float(torch.linalg.norm(fq - fd) / torch.linalg.norm(fd))})
        Q.free()
        del fq
    out["rho_sweep"] = sweep
    print("[bench]   rho sweep: " + ", ".join(f"rho {r['rho']:g}: {r['ms_per_product']:.3f} ms, diff {r['rel_diff_vs_direct']:.2e}"
                                         for r in sweep), file=sys.stderr, flush=True)
    return out


def orth_block(H, torch, np, W, steps=10):
    """Alg. 4.1's QR step and its QRCP truncation on the 64^3 FP64 workload:
    rank, build time, product time and the product's deviation from the
    interpolation form, per stored form."""
    w = W.WORKLOADS["w3d_invr_n64"]
    a = w.a()
    u = torch.tensor(w.rhs(), dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "forms": {}}
    ref = None
    for label, kw in (("interpolation", {}), ("qr", {"orthonormalize": "qr"}),
                      ("qrcp_1e-13", {"orthonormalize": "qrcp"}),
                      ("qrcp_0.3", {"orthonormalize": "qrcp", "rank_tol": 0.3})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = H.htlr_build(None, w.kernel, w.d, w.n, w.p, w.leaf, a=a, precisions=["fp64"], **kw)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        f = M.matvec(u, prec="fp64")
        for _ in range(2):
            M.matvec(u, f, prec="fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            M.matvec(u, f, prec="fp64")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        if ref is None:
            ref = f.clone()
        info = M.info()
        out["forms"][label] = {"rank": info["rank"], "level_rank": info["level_rank"], "build_s": round(build_s, 4),
                               "device_bytes": info["device_bytes"],
                               "ms_per_product": round(ms, 4),
                               "rel_diff_vs_interpolation": float(torch.linalg.norm(f - ref) / torch.linalg.norm(ref))}
        print(f"[bench]   {label}: level ranks {info['level_rank']}, build {build_s:.3f} s, {ms:.3f} ms/product",
              file=sys.stderr, flush=True)
        M.free()
        del f
    return out


def serve_block(H, np, W, count, rates=(0.5,)):
    """Serving: Poisson arrivals of mixed solve requests (d, n, kernel, p drawn
    per request, f ~ N(0,1), a = 1 + x_1/2, relative residual 1e-8 in FP64).
    Capacity with bfloat16-core, FP32 and FP64 inner products (the first two
    refined in FP64 to the same residual); the arrival-rate sweep with
    bfloat16-core inner products, the fastest served form."""
    A = {}

    def a_of(d, n):
        if (d, n) not in A:
            A[(d, n)] = 1.0 + 0.5 * W.grid_points([W.uniform_nodes(n)] * d)[:, 0]
        return A[(d, n)]

    def drain(S, pending):
        done = {}
        while pending:
            S.step()
            for rid in list(pending):
                u, info = S.result(rid)
                if u is not None or info["state"] >= 2:
                    done[rid] = info
                    pending.discard(rid)
        return done

    def run(S, reqs, fs, times):
        """Submit request i at server time t0 + times[i]; step until done."""
        t0 = S.clock()
        pending, done, order = set(), {}, list(range(len(reqs)))
        arrival = {}
        i = 0
        while i < len(order) or pending:
            now = S.clock() - t0
            while i < len(order) and times[order[i]] <= now:
                r = reqs[order[i]]
                rid = S.submit(fs[order[i]], r.kernel, r.d, r.n, r.p, 8, a=a_of(r.d, r.n), tol=1e-8)
                arrival[rid] = t0 + times[order[i]]
                pending.add(rid)
                i += 1
            if not pending:
                time.sleep(max(0.0, min(0.01, times[order[i]] - now)))
                continue
            S.step()
            for rid in list(pending):
                u, info = S.result(rid)
                if u is not None or info["state"] >= 2:
                    info["latency"] = info["t_done"] - arrival[rid]
                    done[rid] = info
                    pending.discard(rid)
        span = S.clock() - t0
        lat = sorted(v["latency"] for v in done.values())
        return {"requests": len(done), "makespan_s": round(span, 3), "solves_per_s": round(len(done) / span, 3),
                "p50_latency_s": round(lat[len(lat) // 2], 4), "p99_latency_s": round(lat[int(0.99 * (len(lat) - 1))], 4),
                "max_rel_residual": max(v["rel_residual"] for v in done.values()),
                "all_converged": all(v["status"] == 0 for v in done.values())}

    reqs = W.request_stream(count, rate=1.0)
    fs = [r.rhs() for r in reqs]
    out = {"requests": count, "tol": 1e-8, "max_active": 256, "max_batch": 16}
    for inner in ("bf16", "fp32", "fp64"):
        S = H.Server(max_active=256, max_batch=16, inner_prec=inner, use_graphs=True)
        seen = {}
        for r in reqs:
            seen.setdefault((r.d, r.n, r.kernel, r.p), r)
        t0 = time.time()
        drain(S, {S.submit(r.rhs(), r.kernel, r.d, r.n, r.p, 8, a=a_of(r.d, r.n), tol=1e-8) for r in seen.values()})
        warm = time.time() - t0
        cap = run(S, reqs, fs, [0.0] * count)
        res = {"structures": len(seen), "warm_build_s": round(warm, 2), "capacity": cap}
        if inner == "bf16":
            res["rates"] = []
            for x in rates:
                rate = x * cap["solves_per_s"]
                times = [r.arrival / rate for r in reqs]       # request_stream uses unit rate
                res["rates"].append(dict(run(S, reqs, fs, times), x_capacity=x, rate_per_s=round(rate, 3)))
                print(f"[bench]   {x:g} x capacity: {res['rates'][-1]['solves_per_s']} solves/s, "
                      f"p50 {res['rates'][-1]['p50_latency_s']} s, p99 {res['rates'][-1]['p99_latency_s']} s",
                      file=sys.stderr, flush=True)
        st = S.stats()
        res["server"] = {k: st[k] for k in ("ticks", "fused_products", "graph_launches", "group_products",
                                            "grouped_launches", "resident_structures", "resident_bytes")}
        S.close()
        out[f"inner_{inner}"] = res
    return out


def summarize_profile(d, command, workload, prec):
    """Markdown summary of rocprofv3 CSV output: kernel statistics plus HBM
    traffic from FETCH_SIZE / WRITE_SIZE, each calibrated by the counter value
    of the run's 1 GiB device copy (largest copy dispatch)."""
    import csv
    import glob

    def rows(sub, name):
        f = glob.glob(os.path.join(d, sub, "**", name), recursive=True)
        return list(csv.DictReader(open(f[0]))) if f else []

    def short(k):
        k = k.replace("(anonymous namespace)::", "")
        return k.split("(")[0].replace("void ", "")[:70]

    lines = [f"# rocprofv3 summary: {workload}, {prec}", "", "Command:", "", "```", command, "```", ""]
    st = rows("stats", "*kernel_stats.csv")
    lines += ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in st[:14]:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['TotalDurationNs'])/1e6:.2f} | {float(r['Percentage']):.1f} |")
    # per launch by position in the product: a serially issued product runs
    # the levels in ascending order, so the k-th launch of a kernel within
    # each product is the same level every time (products are counted by the
    # near-field launches, one per product: its own kernel, or the leaf
    # gather of the near field on the core apply)
    tr = rows("stats", "*kernel_trace.csv")
    skip = ("build", "near_block", "downcast", "diag", "core_mode", "rocclr")
    seq = [r for r in sorted(tr, key=lambda r: int(r["Dispatch_Id"]))
           if "htlr" in r["Kernel_Name"] and not any(x in r["Kernel_Name"] for x in skip)]
    nprod = sum(1 for r in seq if ("k_near" in r["Kernel_Name"] or "k_leaf_gather" in r["Kernel_Name"])
                and "reduce" not in r["Kernel_Name"])
    if nprod:
        per = {}
        for r in seq:
            per.setdefault(short(r["Kernel_Name"]), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        lines += ["", f"Per launch by position in the product ({nprod} products; levels issued in ascending order):", "",
                  "| kernel | launch in product | launches | avg us |", "|---|---|---|---|"]
        for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
            c = len(v) // nprod if len(v) % nprod == 0 else 0
            if c == 0:
                lines.append(f"| {k} | all | {len(v)} | {sum(v) / len(v):.1f} |")
                continue
            for pos in range(c):
                w = v[pos::c]
                lines.append(f"| {k} | {pos + 1} of {c} | {len(w)} | {sum(w) / len(w):.1f} |")
    traffic = {}
    for sub, name in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        cc = rows(sub, "*counter_collection.csv")
        if not cc:
            continue
        # the largest runtime copy dispatch is the 1 GiB calibration copy
        copies = [float(r["Counter_Value"]) for r in cc if "copybuffer" in r["Kernel_Name"].lower()]
        cal = (1 << 20) / max(copies) if copies else 1.0          # KiB expected for 1 GiB / KiB counted
        agg = {}
        for r in cc:
            agg.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        lines += ["", f"{name} per dispatch (KiB as counted; calibration factor {cal:.3f} from the 1 GiB copy):", "",
                  "| kernel | dispatches | mean KiB | max KiB | calibrated max GB |", "|---|---|---|---|---|"]
        for k, v in sorted(agg.items(), key=lambda kv: -max(kv[1]))[:10]:
            lines.append(f"| {k} | {len(v)} | {sum(v)/len(v):.0f} | {max(v):.0f} | {max(v)*cal*1024/1e9:.3f} |")
            traffic.setdefault(k, {})[name] = max(v) * cal * 1024
    fam = {}
    for k, v in traffic.items():
        key = "near" if "near" in k else ("core" if "core" in k else None)
        if key and "FETCH_SIZE" in v and "WRITE_SIZE" in v:
            b = v["FETCH_SIZE"] + v["WRITE_SIZE"]
            if b > fam.get(key, {}).get("hbm_bytes_per_launch", -1):
                fam[key] = {"kernel": k, "hbm_bytes_per_launch": b, "fetch_bytes": v["FETCH_SIZE"],
                            "write_bytes": v["WRITE_SIZE"]}
    return "\n".join(lines) + "\n", fam


def summarize_counters(d, command, workload, prec):
    """Markdown summary of rocprofv3 SQ counter passes (CSV under d/p1, d/p2):
    per kernel, MFMA and VALU utilisation against the chip's issue capacity.
    Kernel cycles = GRBM_GUI_ACTIVE / 8 (the counter is summed over the 8
    XCDs); 1024 SIMDs; an f64 16x16x4 MFMA keeps its SIMD's matrix pipe busy
    64 cycles (SQ_VALU_MFMA_BUSY_CYCLES reads exactly that times
    SQ_INSTS_MFMA); a wave64 VALU instruction issues over 4 cycles."""
    import csv
    import glob
    from collections import defaultdict
    vals = defaultdict(lambda: defaultdict(list))
    for sub in ("p1", "p2"):
        for f in glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                k = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")[:60]
                vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = [f"# rocprofv3 SQ counters: {workload}, {prec}", "", "Commands:", "", "```", command, "```", "",
             "| kernel | dispatches | kernel us | MFMA busy | VALU busy | VALU instr / MFMA | LDS bank-conflict "
             "cycles / LDS instr | waves |", "|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(vals.items(), key=lambda kv: -sum(kv[1].get("GRBM_GUI_ACTIVE", [0]))):
        if "GRBM_GUI_ACTIVE" not in v or "SQ_INSTS_VALU" not in v:
            continue
        n = len(v["GRBM_GUI_ACTIVE"])
        cyc = sum(v["GRBM_GUI_ACTIVE"]) / n / 8
        mf = sum(v.get("SQ_VALU_MFMA_BUSY_CYCLES", [0])) / n
        mi = sum(v.get("SQ_INSTS_MFMA", [0])) / n
        va = sum(v["SQ_INSTS_VALU"]) / n - mi
        li = sum(v.get("SQ_INSTS_LDS", [0])) / n
        bc = sum(v.get("SQ_LDS_BANK_CONFLICT", [0])) / n
        wv = sum(v.get("SQ_WAVES", [0])) / n
        cap = cyc * 1024
        lines.append(f"| {k} | {n} | {cyc / 2400:.1f} | {100 * mf / cap:.1f}% | {100 * 4 * va / cap:.1f}% | "
                     f"{(va / mi) if mi else float('nan'):.2f} | {(bc / li) if li else 0:.2f} | {wv:.0f} |")
    return "\n".join(lines) + "\n"


def _short(block, keys):
    return {k: block[k] for k in keys if k in block}


def main():
    args = parse()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.cpu_pick, args.cpu_out)
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.profile_command, args.workload, args.prec or ""))
        return
    if args.summarize_profile:
        md, fam = summarize_profile(args.summarize_profile, args.profile_command, args.workload, args.prec or "")
        print(md)
        if args.write_traffic:
            with open(os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{args.prec}.json"), "w") as fh:
                json.dump({"source_digest": source_digest(), "workload": args.workload, "prec": args.prec,
                           "kernels": fam}, fh, indent=1)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import htlr_workloads as W
    import paper_2508_05958_amd as H

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = W.WORKLOADS[args.workload]
    prec = args.prec
    # the headline runs the built-in kernel choices unless --tune; the n = 64
    # block reads the committed tuner cache
    saved_cache = os.environ.pop("HTLR_TUNE_CACHE", None)
    print(f"[bench] {w.name} {prec}: build + {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    t0 = time.time()
    M = build_workload(H, np, w)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    u_host = w.rhs() if w.grid == "uniform" else W.solve_target(w.points())
    u64 = to_device(torch, u_host, torch.float64)
    uh = u64 if prec == "fp64" else u64.float().t().contiguous().t() if u64.dim() == 2 else u64.float()
    M, info, f, nrhs, ms, prof, _ = run_workload(H, torch, w, prec, args.steps, args.warmup, args.prof_steps,
                                                 tune=args.tune, serial=args.serial, M=M, ut=uh)
    value = w.N * nrhs / (ms * 1e-3) / 1e9
    roof, per = roofline(info, w, prec, nrhs, prof, ms, w.name)
    f_ref = f.double() if prec != "fp64" else f
    f_host = f_ref.detach().cpu().numpy()
    dense_fs = {prec: f}
    detail = {"headline": {"workload": w.name, "prec": prec, "ms_per_step": ms, "kernels": per, "roofline": roof,
                           "build_s": build_s, "device_bytes": info["device_bytes"]}}
    out = {
        "metric": METRIC, "value": round(value, 6), "unit": "Gpt/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16-core/f32"}[prec],
        "data": ("synthetic (seeded uniform grid, random u)" if w.grid == "uniform"
                 else "synthetic (warped tensor grid, u = u*(x))"),
        "config": {"workload": w.name, "d": w.d, "n": w.n, "N": w.N, "kernel": KERNEL_LABEL.get(w.kernel, w.kernel),
                   "p": w.p, "leaf": w.leaf, "nrhs": nrhs, "precision": prec, "admissibility": "strong, eta=1",
                   "parallelism": "1 GPU", "autotuned": bool(args.tune)},
        "build_s": round(build_s, 3),
        "roofline": roof,
    }
    if not args.no_extra:
        # the same products in the other precisions, on the same matrix and u
        variants = {}
        u32 = u64.float().t().contiguous().t() if u64.dim() == 2 else u64.float()
        for pr in ("fp64", "fp32", "bf16"):
            if pr == prec or (pr == "bf16" and w.grid != "uniform"):
                continue
            print(f"[bench] {w.name} {pr}: 5 timed steps", file=sys.stderr, flush=True)
            _, info3, f3, nr3, ms3, prof3, _ = run_workload(H, torch, w, pr, 5, 1, 2, M=M,
                                                            ut=u64 if pr == "fp64" else u32)
            f3d = f3.double()
            fr = f_ref if prec == "fp64" else f3d
            err = float(torch.linalg.norm(f3d - fr) / torch.linalg.norm(fr))
            r3, per3 = roofline(info3, w, pr, nr3, prof3, ms3, w.name)
            variants[pr] = {"Gpt_s": round(w.N * nr3 / (ms3 * 1e-3) / 1e9, 5), "ms": round(ms3, 3),
                            "err_vs_fp64": float(f"{err:.3g}"), "kernel": r3["kernel"], "frac": r3["frac"],
                            "product_frac": r3["product_frac"]}
            detail[f"headline_{pr}"] = {"ms_per_step": ms3, "kernels": per3, "roofline": r3, "err_vs_fp64": err}
            dense_fs[pr] = f3
            del f3d
        if w.grid == "uniform":
            # Alg. 4.1's QR step with QRCP truncation at pivot tolerance 0.1:
            # each level keeps its own rank (here the finest level drops below p)
            print(f"[bench] {w.name} fp64, QRCP-truncated factors (rank_tol 0.1): 5 timed steps", file=sys.stderr,
                  flush=True)
            Mq = H.htlr_build(None, w.kernel, w.d, w.n, w.p, w.leaf, a=w.a(), precisions=["fp64"],
                              orthonormalize="qrcp", rank_tol=0.1)
            _, infq, fq, nrq, msq, profq, _ = run_workload(H, torch, w, "fp64", 5, 1, 2, M=Mq, ut=u64)
            err = float(torch.linalg.norm(fq - f_ref) / torch.linalg.norm(f_ref))
            rq, perq = roofline(infq, w, "fp64", nrq, profq, msq, w.name + "_qrcp")
            variants["fp64_qrcp_0.1"] = {"Gpt_s": round(w.N * nrq / (msq * 1e-3) / 1e9, 5), "ms": round(msq, 3),
                                         "level_rank": infq["level_rank"], "err_vs_interpolation": float(f"{err:.3g}"),
                                         "kernel": rq["kernel"], "frac": rq["frac"], "product_frac": rq["product_frac"]}
            detail["headline_fp64_qrcp_0.1"] = {"ms_per_step": msq, "kernels": perq, "roofline": rq,
                                                "level_rank": infq["level_rank"], "err_vs_interpolation": err}
            dense_fs["fp64_qrcp_0.1"] = fq
            Mq.free()
        out["variants"] = variants
    # every product of this block against the dense operator on 1000 seeded rows
    e_dense = dense_row_errors(M, torch, w, u64, dense_fs)
    out["e_apply_rand"] = e_dense
    detail["headline"]["e_apply_rand"] = e_dense
    print(f"[bench]   e_apply;rand on 1000 rows (vs the uncompressed operator): {e_dense}", file=sys.stderr, flush=True)
    del dense_fs
    M.free()
    del f, f_ref, uh, u64
    torch.cuda.empty_cache()
    if saved_cache is not None:
        os.environ["HTLR_TUNE_CACHE"] = saved_cache
    elif args.tune_cache and os.path.exists(args.tune_cache):
        os.environ["HTLR_TUNE_CACHE"] = args.tune_cache
    if args.copy_probe_mib:
        # a plain device-to-device copy of known size (the HIP runtime's copy
        # kernel), used to calibrate the FETCH_SIZE / WRITE_SIZE counters
        import ctypes
        nbytes = args.copy_probe_mib * (1 << 20)
        x = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        assert hip.hipMemcpy(y.data_ptr(), x.data_ptr(), nbytes, 3) == 0      # hipMemcpyDeviceToDevice
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
        del x, y
    if not args.no_small:
        ws = W.WORKLOADS["w3d_invr_n64"]
        print(f"[bench] {ws.name} fp64 (tuner cache)", file=sys.stderr, flush=True)
        M2, info2, f2, nr2, ms2, prof2, b2 = run_workload(H, torch, ws, "fp64", 20, 5, 5, tune=True)
        r2, per2 = roofline(info2, ws, "fp64", nr2, prof2, ms2, ws.name)
        out[ws.name] = {"Gpt_s": round(ws.N / (ms2 * 1e-3) / 1e9, 5), "ms": round(ms2, 4), "kernel": r2["kernel"],
                        "frac": r2["frac"], "product_frac": r2["product_frac"]}
        detail[ws.name] = {"ms_per_step": ms2, "kernels": per2, "roofline": r2}
        M2.free()
        del f2
        torch.cuda.empty_cache()
    if not args.no_tables:
        print("[bench] construction at the paper's table shapes", file=sys.stderr, flush=True)
        tb = paper_tables_block(H, torch, np)
        detail["paper_tables"] = tb
        out["paper_tables"] = {"rows": len(tb["rows"]),
                               "t_c_s_max": max(r["t_c_s"] for r in tb["rows"]),
                               "matvec_ms_max": max(r["matvec_ms"] for r in tb["rows"]),
                               "e_apply_rand_over_paper_max": round(max(r["e_apply_rand"] / r["paper_e_apply_rand"]
                                                                        for r in tb["rows"]), 2)}
        torch.cuda.empty_cache()
    if not args.no_orth:
        print("[bench] orthonormal and QRCP-truncated forms (Alg. 4.1 QR step)", file=sys.stderr, flush=True)
        ob = orth_block(H, torch, np, W)
        detail["w3d_invr_n64_orth"] = ob
        out["orth"] = {k: {"level_rank": v["level_rank"], "ms": v["ms_per_product"]} for k, v in ob["forms"].items()}
        torch.cuda.empty_cache()
    if not args.no_quasi:
        print("[bench] quasi-uniform grid through a uniform one (T Ahat S)", file=sys.stderr, flush=True)
        qb = quasi_block(H, torch, np, W)
        detail["wq2d_log_n512_m1024"] = qb
        out["quasi"] = {"fp64_ms": qb["fp64"]["ms_per_product"], "fp32_ms": qb["fp32"]["ms_per_product"],
                        "Gpt_s_fp64": qb["fp64"]["Gpt_s"], "direct_ms": qb["direct_tensor_grid_ms"]}
        torch.cuda.empty_cache()
    if not args.no_solve:
        print("[bench] warped-grid solve (FP32-IR and FP64 GMRES)", file=sys.stderr, flush=True)
        sb = solve_block(H, torch, np, W)
        detail["w3d_exp_warp_n96_solve"] = sb
        out["solve"] = {"fp32_ir_s": sb["inner_fp32"]["seconds"], "fp64_s": sb["inner_fp64"]["seconds"],
                        "fp32_product_ms": sb["products"]["fp32"]["ms"],
                        "fp32_core_frac": sb["products"]["fp32"]["roofline"]["frac"],
                        "solves_per_s": sb["inner_fp32"]["solves_per_s"],
                        "res": float(f"{sb['inner_fp32']['rel_residual_fp64']:.3g}"),
                        "err_ustar": float(f"{sb['inner_fp32']['rel_err_vs_ustar']:.3g}")}
        torch.cuda.empty_cache()
    if not args.no_serve:
        print(f"[bench] serving: {args.serve_requests} mixed requests (rate sweep with bfloat16-core inner products)", file=sys.stderr, flush=True)
        vb = serve_block(H, np, W, args.serve_requests, [float(x) for x in args.serve_rates.split(",") if x])
        detail["serving"] = vb
        cap = vb["inner_bf16"]["capacity"]
        out["serving"] = {"requests": vb["requests"], "inner": "bf16-core, FP64 refinement",
                          "solves_per_s": cap["solves_per_s"],
                          "p50_s": cap["p50_latency_s"], "p99_s": cap["p99_latency_s"],
                          "fp32_inner_solves_per_s": vb["inner_fp32"]["capacity"]["solves_per_s"],
                          "fp64_inner_solves_per_s": vb["inner_fp64"]["capacity"]["solves_per_s"],
                          "rates": [_short(r, ("x_capacity", "solves_per_s", "p50_latency_s", "p99_latency_s"))
                                    for r in vb["inner_bf16"].get("rates", [])]}
        torch.cuda.empty_cache()
    if not args.no_cpu:
        print(f"[bench] cpu_baseline: oracle on {args.cpu_leaves} leaves of {w.name}", file=sys.stderr, flush=True)
        cb, err = cpu_baseline(w, args.cpu_leaves, args.cpu_procs, f_host)
        out["cpu_baseline"] = cb
        out["err_vs_oracle_sampled"] = float(f"{err:.3g}")
    else:
        out["cpu_baseline"] = None
    print("[bench-detail] " + json.dumps(detail), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
