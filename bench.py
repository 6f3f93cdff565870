"""Throughput of the full Yin-Yang potential solve on one MI355X.

One step = one full solve (angular analysis, radial scans, synthesis on both
patches, plus the operand splits of the reduced precisions) of a synthetic,
device-resident density; plans and autotuning happen before timing.  Prints
one JSON line: the headline's cells/s as `value` (by default the FP64
separable solve), and every method / precision's rate and error against the
FP64 oracle under `precisions` (dense FP64, FP32, BF16x3, FP16x2 and the
separable FP64 form).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload binary]
                    [--precision fp64] [--no-cpu-baseline] [--no-check]
    python bench.py --workload batch64      # 64 uneven fields, batched vs sequential
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
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 6, "fp16x2": 3}   # MFMA products per algorithmic multiply-add
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "fp16x2": "f16x2"}
ALL_PRECISIONS = ("fp64", "fp32", "bf16x3", "fp16x2")
SEP_LP = ("fp32", "bf16x3")   # reduced precisions of the separable form's phi transforms
# every source a timed kernel is compiled from: counter figures taken on other sources are not used
KERNEL_SRCS = [os.path.join(ROOT, "paper_1806_04593_amd", "csrc", f)
               for f in ("yyg_internal.h", "yyg_tile.h", "yyg_kernels.hip", "yyg_kernels_x4.hip",
                         "yyg_kernels_sep_lp.hip", "yyg_kernels_lp.hip", "yyg_batch_sep.hip", "yyg_phi_stream.hip")]
METRIC = "grid cells/sec per full Phi solve, FP64 vs split-precision, at stated max rel. error"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, key, kernel, name=None, tile=None):
    """HBM bytes per launch of one kernel from committed rocprofv3 --pmc
    counters (FETCH_SIZE + WRITE_SIZE, scaled by a calibration kernel of
    known size), or None when absent, taken on different kernel sources or
    on another kernel variant than the one timed (given `name`, the exact
    symbol, also looked up among the per-variant figures; given `tile`, the
    (rows, columns) of a dense GEMM tile)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
        rec = data.get(f"{workload}/{key}")
        if not rec or rec.get("kernel_sha") != kernel_sha():
            return None
        k = rec["kernels"].get(kernel, {})
        if name is not None and k.get("name") != name:
            # not the pinned run's variant: every variant the autotuner
            # launched in an unpinned counter run
            if name in rec.get("by_name", {}):
                return float(rec["by_name"][name]["bytes_per_launch"])
            return None
        if tile is not None:
            args = [int(x) for x in k["name"][k["name"].index("<") + 1:].rstrip(">").split(",")]
            if (args[1], args[2]) != tuple(tile) or "write_kernel" in k:
                return None
        return float(k["bytes_per_launch"])
    except (OSError, ValueError, KeyError, TypeError):
        return None


class OracleFront:
    """The oracle's density-dependent front of a solve (moments of Eqs. 26-27
    and radial sums of Eqs. 19-20, in full), kept for sampled synthesis:
    the error of every measured precision and the CPU baseline use it."""

    def __init__(self, desc, rho):
        import numpy as np
        import oracle as O
        self.desc, self.np = desc, np
        self.polar = desc.get("kind") == "polar"
        self.P = 1 if self.polar else 2
        if self.polar:
            th, ph = O.polar_edges(desc["n_theta"], desc["n_phi"])
            w = np.ones((desc["n_theta"], desc["n_phi"]))
        else:
            th, ph = O.patch_edges(desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"])
            w = O.overlap_weights(th, ph, desc["delta_theta"], desc["delta_phi"])
        T = O.theta_integrals(th, desc["lmax"])
        C, S = O.phi_integrals(ph, desc["lmax"])
        c0, t0 = time.process_time(), time.perf_counter()
        AC, AS = O.moments(rho, w, T, C, S)
        self.UC, self.US = O.radial_sums(AC, AS, desc["r_edges"])
        self.front_s = time.perf_counter() - t0
        self.front_cpu_s = time.process_time() - c0
        self.tc, self.pc = 0.5 * (th[:-1] + th[1:]), 0.5 * (ph[:-1] + ph[1:])

    def at(self, s):
        """Phi at samples s[:, (p, n, j, k)]."""
        import oracle as O
        t, f = self.tc[s[:, 2]], self.pc[s[:, 3]]
        if self.polar:
            return O.potential_polar_at(self.UC, self.US, self.desc["G"], s[:, 1], t, f)
        return O.potential_at(self.UC, self.US, self.desc["G"], s[:, 0], s[:, 1], t, f)

    def samples(self, k, seed):
        np = self.np
        d = self.desc
        nR = len(d["r_edges"]) - 1
        rng = np.random.default_rng(seed)
        return np.stack([rng.integers(0, self.P, k), rng.integers(0, nR, k), rng.integers(0, d["n_theta"], k),
                         rng.integers(0, d["n_phi"], k)], 1)


_FRONT = None   # the oracle front shared with forked baseline workers


def _synth_chunks(args):
    """Baseline worker: synthesise `n` chunks of `pts` consecutive angular
    cells of a random (patch, shell) row each, as the oracle's full solve
    does row by row; returns the outputs done and the wall seconds."""
    import numpy as np
    n, pts, seed = args
    d = _FRONT.desc
    nang = d["n_theta"] * d["n_phi"]
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    for i in range(n):
        a0 = int(rng.integers(0, max(1, nang - pts + 1)))
        a = np.arange(a0, min(nang, a0 + pts))
        s = np.stack([np.full(a.size, rng.integers(0, _FRONT.P)), np.full(a.size, rng.integers(0, len(d["r_edges"]) - 1)),
                      a // d["n_phi"], a % d["n_phi"]], 1)
        _FRONT.at(s)
    return n * pts, time.perf_counter() - t0


def cpu_baseline(front, budget_s=10.0, pts=4096):
    """The oracle as it stands, timed on this host: its front (moments and
    radial sums, in full) as computed for the error checks, then its
    synthesis of whole chunks of outputs, on every available core at once
    (one forked process per core, each synthesising independent chunks)
    and on one core.  The full solve's time is the front plus the synthesis
    of every output at the measured rate (extrapolated)."""
    import multiprocessing as mp
    global _FRONT
    _FRONT = front
    d = front.desc
    cells = front.P * (len(d["r_edges"]) - 1) * d["n_theta"] * d["n_phi"]
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    # one core: chunks until about a third of the budget
    done, t1 = 0, time.perf_counter()
    i = 0
    while time.perf_counter() - t1 < budget_s / 3 or done == 0:
        done += _synth_chunks((1, pts, 10_000 + i))[0]
        i += 1
    rate1 = done / (time.perf_counter() - t1)
    per = max(1, int(round(rate1 * (2 * budget_s / 3) / pts)))   # chunks per worker
    ctx = mp.get_context("fork")
    t2 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_synth_chunks, [(per, pts, w) for w in range(cores)])
    wall = time.perf_counter() - t2
    rate = sum(r[0] for r in res) / wall
    est = front.front_s + cells / rate
    est1 = front.front_s + cells / rate1
    return {"value": cells / est, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": (f"{d['name']}: moments and radial sums in full ({front.front_s:.1f} s, one process), then "
                       f"{cores} processes x {per} chunks of {pts} outputs of the synthesis ({wall:.1f} s); the full "
                       f"solve's {cells:.3g} outputs extrapolated to {est:.0f} s"),
            "single_core": {"value": cells / est1, "cores": 1,
                            "sample": f"{done} outputs synthesised on one core; full solve extrapolated to {est1:.0f} s"},
            "front_s": round(front.front_s, 2), "extrapolated": True}


def sampled_error(front, phi_host, k=400, seed=123):
    import numpy as np
    s = front.samples(k, seed)
    ref = front.at(s)
    got = phi_host[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
    return float(np.max(np.abs(got - ref) / np.abs(ref)))


def timed_steps(g, d_phi, prec, a):
    """Warm-up, then the mean milliseconds of `a.steps` back-to-back solves
    between two events on the current stream (no per-phase events)."""
    import torch
    for _ in range(a.warmup):
        g.solve(d_phi, prec)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(a.steps):
        g.solve(d_phi, prec)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / a.steps


def phase_pass(g, d_phi, prec, a):
    """The same solves again with the library's per-phase HIP events
    (recorded on the solve stream around each phase's launches); returns
    summed milliseconds and launch counts per timing slot."""
    import torch
    g.set_timing(True)
    torch.cuda.synchronize()
    for _ in range(a.steps):
        g.solve(d_phi, prec)
    torch.cuda.synchronize()
    kms, kcnt = g.timing()
    g.set_timing(False)
    return kms, kcnt


def phase_alone_ms(g, d_phi, phase, a):
    """Average duration of one separable phase launched alone, a.steps times
    back to back between two HIP events on the stream it runs on (after a
    solve: each launch recomputes the same output)."""
    import torch
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # warm-up by time (at least 0.2 s of launches), so that the clocks have
    # settled at their loaded level whatever ran before
    t0 = time.perf_counter()
    n = 0
    while n < 3 or time.perf_counter() - t0 < 0.2:
        g.sep_phase(phase, d_phi)
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    start.record()
    for _ in range(a.steps):
        g.sep_phase(phase, d_phi)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / a.steps


# dense autotuning times every tile and split on the plan's shapes; above
# this many cells (the binary workload: 1.97e8) its sweep would take minutes,
# and the dense contractions run their fixed heuristic configuration
DENSE_TUNE_MAX_CELLS = 5e7


def phi_folded(kname):
    """Whether a phi-transform kernel works on the rows folded about the
    central meridian (half the multiply-adds of the unfolded count)."""
    args = kname[kname.find("<") + 1:].rstrip(">").split(", ")
    # the streaming kernels run on mirror-symmetric grids only, always folded
    return bool(kname.startswith(("yyg::phi_syn_lean_kernel<", "yyg::phi_syn_stream", "yyg::phi_ana_stream"))
                or (kname.startswith("yyg::phi_direct_kernel<") and args[-1] == "true")
                or (kname.startswith("yyg::gemm_nt_f64_batched<") and int(args[-1]) & (128 | 256 | 4096)))


def phi_roofline(head, desc, M, nang):
    """Roofline of the dominant single-launch kernel of the separable solve,
    the longer phi transform."""
    k = head["kernels_ms"]
    L2 = 2 * desc["lmax"] + 1
    cand = {
        "phi_analysis": (k["phi_analysis"], 2.0 * M * nang * L2, 8.0 * M * nang + 8.0 * M * desc["n_theta"] * L2),
        "phi_synthesis": (k["phi_synthesis"], 2.0 * M * nang * L2, 8.0 * M * nang + 8.0 * M * desc["n_theta"] * L2),
    }
    name = max(cand, key=lambda n: cand[n][0])
    ms_solve, flops_k, bytes_k = cand[name]
    # the kernel's average duration: launched alone, back to back (the
    # per-phase events inside solves add a launch gap to each)
    ms_k = head["phase_alone_ms"][name]
    kname = head["kernel_names"][name]
    if phi_folded(kname):
        flops_k /= 2.0   # folded about the central meridian: half the multiply-adds
    tf = flops_k / (ms_k * 1e-3) / 1e12
    gbs = bytes_k / (ms_k * 1e-3) / 1e9
    fm, fh = tf / PEAK["fp64"], gbs / 8000.0
    if fm >= fh:
        roof = {"bound": "mfma", "kernel": kname, "achieved": tf, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": fm, "hbm_frac": fh}
    else:
        roof = {"bound": "hbm", "kernel": kname, "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                "frac": fh, "mfma_frac": fm}
    roof["phase"] = name
    roof["ms_per_launch"] = ms_k
    roof["achieved_in_solve"] = (tf if roof["unit"] == "TFLOP/s" else gbs) * ms_k / ms_solve
    roof["algorithmic_flops"] = flops_k
    roof["algorithmic_bytes"] = bytes_k
    return roof, name, kname


def bench_single(a):
    import torch

    from paper_1806_04593_amd import workloads as W
    from paper_1806_04593_amd import yyg

    desc = W.describe(a.workload)
    nR = len(desc["r_edges"]) - 1
    Q = (desc["lmax"] + 1) ** 2
    nang = desc["n_theta"] * desc["n_phi"]
    P = W.n_patches(desc)
    cells = P * nR * nang
    M = P * nR
    log(f"[bench] workload {a.workload}: n_r={nR} {desc['n_theta']}x{desc['n_phi']} lmax={desc['lmax']}")
    rho = W.density(desc)
    # the oracle's front and the CPU baseline run before the GPU is touched
    # (the baseline forks worker processes)
    front = None
    if not (a.no_check and a.no_cpu_baseline):
        log("[bench] oracle: moments and radial sums")
        front = OracleFront(desc, rho)
    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(front)
        log(f"[bench] oracle {cpu['value']:.3e} cells/s on {cpu['cores']} cores")
    t0 = time.perf_counter()
    g = yyg.Grid(desc, 0)
    plan_s = time.perf_counter() - t0
    log(f"[bench] plan built in {plan_s:.2f} s")
    d_rho = torch.from_numpy(rho).to("cuda:0")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda:0")
    g.upload_rho(d_rho)
    results = {}
    sep_head = a.method == "separable" and a.precision == "fp64"

    # separable form (FP64): phi/theta transforms and rotated cross-patch moments
    if sep_head or not a.only:
        g.set_method("separable")
        t0 = time.perf_counter()
        if not a.no_autotune:
            g.autotune("fp64")
        tune_s = time.perf_counter() - t0
        if a.sep_variants:
            # profiling runs: the variants an unprofiled run chose (the
            # autotuner's timings shift under a profiler)
            for phase, v in enumerate(int(x) for x in a.sep_variants.split(",")):
                if v >= 0:
                    g.sep_config(phase, v)
        ms = timed_steps(g, d_phi, "fp64", a)
        kms, kcnt = phase_pass(g, d_phi, "fp64", a)
        avg = [float(kms[i] / max(1, kcnt[i])) for i in range(8)]
        # the phases alone before the host-side error check: the GPU must
        # not sit idle (and clock down) between the solves and these launches
        alone = {n: phase_alone_ms(g, d_phi, ph, a) for n, ph in (("phi_analysis", 0), ("phi_synthesis", 4))}
        err = None if a.no_check else sampled_error(front, d_phi.cpu().numpy())
        L2 = 2 * desc["lmax"] + 1
        phi_flops = 2.0 * M * nang * L2           # each phi transform (unfolded count)
        # algorithmic TFLOP/s of each phi transform in the solve (halved
        # count for the folded kernels)
        names = {p: g.sep_kernel(q) for p, q in (("phi_analysis", 0), ("phi_synthesis", 4))}
        alg = {p: phi_flops / (2.0 if phi_folded(n) else 1.0) for p, n in names.items()}
        results["fp64_separable"] = {
            "cells_per_s": cells / (ms * 1e-3), "ms_per_step": ms, "max_rel_err_vs_oracle": err,
            "kernels_ms": {"phi_analysis": avg[4], "theta_analysis_rotation": avg[5], "radial_scan": avg[1],
                           "theta_synthesis": avg[6], "phi_synthesis": avg[7]},
            "phi_synthesis_tflops": alg["phi_synthesis"] / (avg[7] * 1e-3) / 1e12,
            "phi_analysis_tflops": alg["phi_analysis"] / (avg[4] * 1e-3) / 1e12,
            "phase_alone_ms": alone, "variants": g.sep_info(), "tune_s": round(tune_s, 2),
            "kernel_names": {n: g.sep_kernel(p) for p, n in enumerate(
                ("phi_analysis", "theta_analysis", "rotation", "theta_synthesis", "phi_synthesis"))},
        }
        log(f"[bench] fp64 separable: {ms:.4f} ms/step, {cells / (ms * 1e-3):.3e} cells/s, err {err}, "
            f"kernels {avg[4:]} scan {avg[1]}")
        # the same form with its two phi transforms in FP32 / BF16 x 3
        for prec in ([] if a.only else SEP_LP):
            t0 = time.perf_counter()
            if not a.no_autotune:
                g.autotune(prec)
            tune_s = time.perf_counter() - t0
            ms = timed_steps(g, d_phi, prec, a)
            kms, kcnt = phase_pass(g, d_phi, prec, a)
            avg = [float(kms[i] / max(1, kcnt[i])) for i in range(8)]
            err = None if a.no_check else sampled_error(front, d_phi.cpu().numpy())
            results[f"{prec}_separable"] = {
                "cells_per_s": cells / (ms * 1e-3), "ms_per_step": ms, "max_rel_err_vs_oracle": err,
                "method": "separable", "tune_s": round(tune_s, 2),
                "kernels_ms": {"phi_analysis": avg[4], "theta_analysis_rotation": avg[5], "radial_scan": avg[1],
                               "theta_synthesis": avg[6], "phi_synthesis": avg[7]},
                "kernel_names": {"phi_analysis": g.sep_lp_kernel(prec, 0), "phi_synthesis": g.sep_lp_kernel(prec, 4)},
            }
            log(f"[bench] {prec} separable: {ms:.4f} ms/step, {cells / (ms * 1e-3):.3e} cells/s, err {err}, "
                f"kernels {avg[4:]} scan {avg[1]}")
        g.set_method("dense")

    # dense form: every precision of the two angular contractions
    tune_dense = not a.no_autotune and cells <= DENSE_TUNE_MAX_CELLS
    precisions = [] if (a.only and sep_head) else (
        [a.precision] if a.only else [a.precision] + [p for p in ALL_PRECISIONS if p != a.precision])
    for prec in precisions:
        t0 = time.perf_counter()
        g.prepare(prec)
        if tune_dense:
            g.autotune(prec)
        tune_s = time.perf_counter() - t0
        info = g.plan_info(prec)
        ms = timed_steps(g, d_phi, prec, a)
        kms, kcnt = phase_pass(g, d_phi, prec, a)
        avg = [float(kms[i] / max(1, kcnt[i])) for i in range(4)]
        err = None if a.no_check else sampled_error(front, d_phi.cpu().numpy())
        flops_syn = 2.0 * M * nang * (P * Q)
        achieved = flops_syn / (avg[2] * 1e-3) / 1e12
        results[prec] = {"cells_per_s": cells / (ms * 1e-3), "ms_per_step": ms, "max_rel_err_vs_oracle": err,
                         "method": "dense", "autotuned": tune_dense,
                         "kernels_ms": {"analysis": avg[0], "radial_scan": avg[1], "synthesis": avg[2],
                                        "operand_split": avg[3]},
                         "synthesis_tflops": achieved, "launch": info, "prepare_tune_s": round(tune_s, 2)}
        log(f"[bench] dense {prec}: {ms:.4f} ms/step, {cells / (ms * 1e-3):.3e} cells/s, err {err}, kernels {avg}")

    # speed-ups against the fastest FP64 form (and against dense FP64)
    fp64_forms = [results[k]["ms_per_step"] for k in ("fp64_separable", "fp64") if k in results]
    best64 = min(fp64_forms) if fp64_forms else None
    for key, r in results.items():
        r["speedup_vs_fastest_fp64"] = best64 / r["ms_per_step"] if best64 else None
        r["speedup_vs_dense_fp64"] = results["fp64"]["ms_per_step"] / r["ms_per_step"] if "fp64" in results else None

    head_key = "fp64_separable" if sep_head else a.precision
    head = results[head_key]

    def dense_roofline(prec):
        r = results[prec]
        ach = r["synthesis_tflops"]
        pk = PEAK[prec]
        return {"bound": "mfma",
                "kernel": ("gemm_nt_f64_kernel<1,...> (dense synthesis)" if prec == "fp64"
                           else f"gemm_nt_lp_kernel<1,{prec},...> (dense synthesis)"),
                "achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk,
                "traffic": measured_traffic(a.workload, prec, "synthesis",
                                            tile=(r["launch"]["bm_syn"], r["launch"]["bn_syn"])),
                "executed_products_per_mac": PRODUCTS[prec], "executed_frac": ach * PRODUCTS[prec] / pk}

    if head_key == "fp64_separable":
        roof, name, kname = phi_roofline(head, desc, M, nang)
        roof["traffic"] = measured_traffic(a.workload, head_key, name, kname)
    else:
        roof = dense_roofline(head_key)
    out = {
        "metric": METRIC,
        "value": head["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.precision],
        "data": "synthetic",
        "config": {"workload": a.workload, "grid": desc.get("kind", "yinyang"), "patches": P, "n_r": nR,
                   "n_theta": desc["n_theta"], "n_phi": desc["n_phi"],
                   "lmax": desc["lmax"], "cells": cells, "precision": a.precision,
                   "method": "separable" if head_key == "fp64_separable" else "dense",
                   "max_rel_err_vs_oracle": head["max_rel_err_vs_oracle"], "plan_build_s": round(plan_s, 3)},
        "roofline": roof,
        "roofline_dense_fp64": dense_roofline("fp64") if "fp64" in results else None,
        "kernels_ms": head["kernels_ms"],
        "precisions": results,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_batch(a):
    import numpy as np
    import torch

    from paper_1806_04593_amd import workloads as W
    from paper_1806_04593_amd import yyg

    descs = W.batch_descs(64)
    cells = sum(2 * (len(d["r_edges"]) - 1) * d["n_theta"] * d["n_phi"] for d in descs)
    flops_syn = sum(2.0 * 2 * (len(d["r_edges"]) - 1) * d["n_theta"] * d["n_phi"] * 2 * (d["lmax"] + 1) ** 2
                    for d in descs)
    log(f"[bench] batch64: {len(descs)} fields, {cells} cells")
    rhos = [W.density(d) for d in descs]
    check = (0, 21, 42, 63)
    fronts = {} if a.no_check else {i: OracleFront(descs[i], rhos[i]) for i in check}
    t0 = time.perf_counter()
    grids = [yyg.Grid(d, 0) for d in descs]
    plan_s = time.perf_counter() - t0
    log(f"[bench] 64 plans built in {plan_s:.1f} s")
    d_rho = [torch.from_numpy(r).to("cuda:0") for r in rhos]
    d_phi = [torch.empty(g.shape, dtype=torch.float64, device="cuda:0") for g in grids]
    stream = torch.cuda.Stream()
    for g, r in zip(grids, d_rho):
        g.upload_rho(r)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(a.steps):
            fn()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / a.steps

    def errors():
        if a.no_check:
            return None
        return max(sampled_error(fronts[i], d_phi[i].cpu().numpy(), k=100, seed=i) for i in check)

    def seq():
        for g, p in zip(grids, d_phi):
            g.solve(p, "fp64", stream=stream)

    # 64 sequential FP64 solves in each form, each plan autotuned on its own shape
    sequential = {}
    for method in ("dense", "separable"):
        for g in grids:
            g.set_method(method)
            if not a.no_autotune:
                g.autotune("fp64")
        sequential[method] = timed(seq)
        log(f"[bench] 64 sequential {method} FP64 solves: {sequential[method]:.3f} ms")
    seq_best = min(sequential.values())

    results = {}
    forms = [("fp64_separable", "fp64", "separable")] + [(p, p, "dense") for p in ALL_PRECISIONS]
    if a.only:
        forms = [f for f in forms if f[0] == ("fp64_separable" if a.method == "separable" and a.precision == "fp64"
                                               else a.precision)]
    for key, prec, method in forms:
        for g in grids:
            g.set_method(method)
            g.prepare(prec)
        b = yyg.Batch(grids, prec)
        b.solve(d_rho, d_phi, stream=stream)
        stream.synchronize()
        if not a.no_autotune:
            b.autotune(stream=stream)
        ms = timed(lambda: b.solve(d_rho, d_phi, stream=stream))
        prof = np.mean([b.profile(stream=stream) for _ in range(3)], axis=0)
        err = errors()
        results[key] = {"cells_per_s": cells / (ms * 1e-3), "ms_per_step": ms, "method": method,
                        "speedup_vs_sequential_fastest_fp64": seq_best / ms,
                        "speedup_vs_sequential_dense_fp64": sequential["dense"] / ms,
                        "speedup_vs_sequential_separable_fp64": sequential["separable"] / ms,
                        "max_rel_err_vs_oracle": err,
                        "kernels_ms": {"analysis": prof[0], "radial_scan": prof[1], "synthesis": prof[2],
                                       "operand_split": prof[3]},
                        "batch": b.info()}
        if method == "dense":
            results[key]["synthesis_tflops"] = flops_syn / (prof[2] * 1e-3) / 1e12
        log(f"[bench] batched {key}: {ms:.3f} ms ({seq_best / ms:.2f}x the fastest sequential FP64), "
            f"phases {prof}, err {err}")
        b.close()
    head_key = "fp64_separable" if (a.method == "separable" and a.precision == "fp64") else a.precision
    head = results[head_key]
    if head["method"] == "dense":
        ach = head["synthesis_tflops"]
        roof = {"bound": "mfma", "kernel": f"gemm grouped synthesis ({a.precision})", "achieved": ach,
                "peak": PEAK[a.precision], "unit": "TFLOP/s", "frac": ach / PEAK[a.precision], "traffic": None,
                "executed_products_per_mac": PRODUCTS[a.precision],
                "executed_frac": ach * PRODUCTS[a.precision] / PEAK[a.precision]}
    else:
        # grouped phi transforms: FP64 flops of the folded transforms over their phases' time
        fl = sum(2.0 * 2 * (len(d["r_edges"]) - 1) * d["n_theta"] * d["n_phi"] * (2 * d["lmax"] + 1) / 2
                 for d in descs)
        t = (head["kernels_ms"]["analysis"] + head["kernels_ms"]["synthesis"]) * 1e-3
        roof = {"bound": "mfma", "kernel": "grouped separable phases (both phi transforms and theta phases)",
                "achieved": fl / t / 1e12, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": fl / t / 1e12 / PEAK["fp64"], "traffic": None}
    out = {
        "metric": METRIC, "value": head["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[a.precision], "data": "synthetic",
        "config": {"workload": "batch64", "fields": len(descs), "cells": cells, "precision": a.precision,
                   "method": head["method"],
                   "sequential_fp64_ms": sequential, "max_rel_err_vs_oracle": head["max_rel_err_vs_oracle"],
                   "plan_build_s": round(plan_s, 2)},
        "roofline": roof,
        "precisions": results,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="binary")
    ap.add_argument("--precision", default="fp64", choices=ALL_PRECISIONS)
    ap.add_argument("--method", default="separable", choices=("dense", "separable"),
                    help="headline method for FP64 (both are measured unless --only)")
    ap.add_argument("--only", action="store_true", help="measure the headline precision only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--sep-variants", default=None,
                    help="comma-separated variants of the five separable phases (as yyg_sep_config), set after "
                         "autotuning; for profiling the kernels an unprofiled run chose")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {a.gpus} requested): the solver holds the whole grid on "
              "one device and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if a.workload == "batch64":
        bench_batch(a)
    else:
        bench_single(a)


if __name__ == "__main__":
    main()
