"""Throughput of the full Yin-Yang potential solve on one MI355X.

One step = one full solve (angular analysis, radial scans, synthesis on both
patches) of a synthetic, device-resident density; the plan (tables) is built
before timing.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sn_core]
                    [--precision fp64] [--no-cpu-baseline]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x2": 2500.0}   # dense MFMA TFLOP/s
# MFMA products executed per algorithmic multiply-add (operand-split terms)
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 6, "fp16x2": 3}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "fp16x2": "f16x2"}
KERNEL_SRC = os.path.join(ROOT, "paper_1806_04593_amd", "csrc", "yyg_kernels.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload, precision, n_launch_units):
    """HBM bytes per launch of the synthesis kernel from committed rocprofv3
    --pmc counters (FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated), or
    None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
        rec = data.get(f"{workload}/{precision}")
        if not rec or rec.get("kernel_sha") != kernel_sha():
            return None
        return float(rec["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(desc, rho, budget_s=20.0):
    """Oracle (as it stands) on the host: full moments and radial sums, then
    synthesis of a bounded number of (patch, shell) rows, extrapolated to the
    full grid.  Returns the cells/s figure and what was sampled."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    args = (desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"],
            desc["lmax"], desc["G"])
    th, ph = O.patch_edges(*args[1:5])
    tables = (th, ph, O.overlap_weights(th, ph, args[3], args[4]), O.theta_integrals(th, args[5]),
              *O.phi_integrals(ph, args[5]))
    nR = len(desc["r_edges"]) - 1
    nang = desc["n_theta"] * desc["n_phi"]
    c0, t0 = time.process_time(), time.perf_counter()
    AC, AS = O.moments(rho, tables[2], tables[3], tables[4], tables[5])
    UC, US = O.radial_sums(AC, AS, desc["r_edges"])
    t_front = time.perf_counter() - t0
    tc = 0.5 * (th[:-1] + th[1:])
    pc = 0.5 * (ph[:-1] + ph[1:])
    T, P = np.meshgrid(tc, pc, indexing="ij")
    tt, pp = T.ravel(), P.ravel()
    rows = 0
    t1 = time.perf_counter()
    rng = np.random.default_rng(0)
    while rows < 2 * nR:
        p, n = int(rng.integers(2)), int(rng.integers(nR))
        O.potential_at(UC, US, desc["G"], np.full(nang, p), np.full(nang, n), tt, pp)
        rows += 1
        if time.perf_counter() - t1 > budget_s:
            break
    t_rows = time.perf_counter() - t1
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    est = t_front + t_rows / rows * (2 * nR)
    cells = 2 * nR * nang
    return {"value": cells / est, "unit": "cells/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"full moments + radial sums, synthesis of {rows} of {2 * nR} (patch, shell) rows; "
                       f"full-solve time extrapolated to {est:.1f} s"),
            "measured_s": round(wall, 2), "effective_cores": round(cpu / wall, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sn_core")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {a.gpus} requested); the solver holds the whole grid "
              "on one device and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1806_04593_amd import workloads as W
    from paper_1806_04593_amd import yyg

    desc = W.describe(a.workload)
    nR = len(desc["r_edges"]) - 1
    log(f"[bench] workload {a.workload}: n_r={nR} {desc['n_theta']}x{desc['n_phi']} lmax={desc['lmax']} "
        f"precision={a.precision}")
    rho = W.density(desc)
    log("[bench] density generated")
    t0 = time.perf_counter()
    g = yyg.Grid(desc, 0)
    if a.precision != "fp64":
        g.prepare(a.precision)
    plan_s = time.perf_counter() - t0
    log(f"[bench] plan built in {plan_s:.2f} s")
    tune_s = 0.0
    if not a.no_autotune:
        t0 = time.perf_counter()
        g.autotune(a.precision)
        tune_s = time.perf_counter() - t0
    info = g.plan_info(a.precision)
    log(f"[bench] launch configuration {info} (autotune {tune_s:.2f} s)")
    d_rho = torch.from_numpy(rho).to("cuda:0")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda:0")
    g.upload_rho(d_rho)
    for _ in range(a.warmup):
        g.solve(d_phi, a.precision)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    g.set_timing(True)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(a.steps):
        g.solve(d_phi, a.precision)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / a.steps
    kms, kcnt = g.timing()
    g.set_timing(False)
    log(f"[bench] timed {a.steps} steps: {ms:.4f} ms/step")

    Q = (desc["lmax"] + 1) ** 2
    nang = desc["n_theta"] * desc["n_phi"]
    cells = 2 * nR * nang
    M = 2 * nR
    flops_syn = 2.0 * M * nang * (2 * Q)
    flops_ana = 2.0 * M * nang * Q
    avg = [kms[i] / max(1, kcnt[i]) for i in range(4)]
    achieved = flops_syn / (avg[2] * 1e-3) / 1e12
    peak = PEAK[a.precision]
    traffic = measured_traffic(a.workload, a.precision, 1)

    err = None
    if not a.no_check:
        import oracle as O
        rng = np.random.default_rng(123)
        s = np.stack([rng.integers(0, 2, 400), rng.integers(0, nR, 400),
                      rng.integers(0, desc["n_theta"], 400), rng.integers(0, desc["n_phi"], 400)], 1)
        ref = O.solve_sampled(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"],
                              desc["delta_phi"], desc["lmax"], desc["G"], rho, s)
        got = d_phi.cpu().numpy()[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
        err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        log(f"[bench] max rel err vs oracle over 400 sampled cells: {err:.3e}")

    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(desc, rho)
        log(f"[bench] oracle {cpu['value']:.3e} cells/s")

    out = {
        "metric": "grid cells/sec per full Phi solve, FP64 vs split-precision, at stated max rel. error",
        "value": cells / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.precision],
        "data": "synthetic",
        "config": {"workload": a.workload, "n_r": nR, "n_theta": desc["n_theta"], "n_phi": desc["n_phi"],
                   "lmax": desc["lmax"], "cells": cells, "precision": a.precision,
                   "max_rel_err_vs_oracle": err, "plan_build_s": round(plan_s, 3),
                   "autotune_s": round(tune_s, 3), "launch": info},
        "roofline": {"bound": "mfma", "kernel": ("gemm_nt_f64_kernel<1,...> (synthesis)" if a.precision == "fp64"
                                                 else f"gemm_nt_lp_kernel<1,...> (synthesis, {a.precision})"),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic,
                     "executed_products_per_mac": PRODUCTS[a.precision],
                     "executed_frac": achieved * PRODUCTS[a.precision] / peak},
        "kernels_ms": {"analysis": avg[0], "radial_scan": avg[1], "synthesis": avg[2], "convert": avg[3]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
