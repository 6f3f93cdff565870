"""Profiling driver: a known-size elementwise kernel (dst = src + 1 over
--copy-mib MiB: reads and writes exactly that many bytes; the calibration of
hardware byte counters) followed by a few solves of one workload.

    python paper_1806_04593_amd/prof_driver.py --workload sn_core --precision fp64 --method separable --solves 3

Run under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) to read the HBM
bytes of each kernel; the calibration kernel moves exactly --copy-mib MiB each way.
"""

import argparse
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sn_core")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--method", default="dense", choices=("dense", "separable"))
    ap.add_argument("--solves", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--sep-variants", default=None,
                    help="comma-separated variants of the five separable phases (as yyg_sep_config), "
                         "instead of the autotuner's choice, to profile the kernels a bench run chose")
    ap.add_argument("--sep-lp-tiles", default=None,
                    help="analysis,synthesis tiles of the reduced-precision phi transforms (as yyg_sep_lp_config) "
                         "for --precision fp32 / bf16x3 with the separable method")
    ap.add_argument("--dense-config", default=None,
                    help="var_ana,split_ana,var_syn of the dense plan (as yyg_plan_config) instead of the "
                         "autotuner's choice")
    a = ap.parse_args()

    import torch

    from paper_1806_04593_amd import workloads as W
    from paper_1806_04593_amd import yyg

    n = a.copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.add(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"[prof] calibration: read and wrote {a.copy_mib} MiB", flush=True)

    desc = W.describe(a.workload)
    rho = W.density(desc)
    g = yyg.Grid(desc, 0)
    g.prepare(a.precision)
    if a.method == "separable":
        g.set_method("separable")
    if a.sep_variants and a.method == "separable":
        for phase, v in enumerate(int(x) for x in a.sep_variants.split(",")):
            if v >= 0:
                g.sep_config(phase, v)
    elif a.dense_config and a.method == "dense":
        va, sp, vs = (int(x) for x in a.dense_config.split(","))
        g.set_config(va, sp, vs, a.precision)
    else:
        g.autotune(a.precision)
    if a.sep_lp_tiles and a.method == "separable" and a.precision in yyg.PRECISIONS and a.precision != "fp64":
        for phase, t in zip((0, 4), (int(x) for x in a.sep_lp_tiles.split(","))):
            st = yyg.lib().yyg_sep_lp_config(g.handle, yyg.PRECISIONS[a.precision], phase, t)
            if st != 0:
                raise SystemExit(f"yyg_sep_lp_config({a.precision}, {phase}, {t}) returned {st}")
    d_rho = torch.from_numpy(rho).to("cuda:0")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda:0")
    g.upload_rho(d_rho)
    t0 = time.perf_counter()
    for _ in range(a.solves):
        g.solve(d_phi, a.precision)
    torch.cuda.synchronize()
    launch = ([g.sep_kernel(p) for p in range(5)] if a.method == "separable" else g.plan_info(a.precision))
    if a.method == "separable" and a.precision != "fp64":
        launch += [g.sep_lp_kernel(a.precision, 0), g.sep_lp_kernel(a.precision, 4)]
    print(f"[prof] {a.solves} solves of {a.workload} ({a.precision}, {a.method}) in {time.perf_counter() - t0:.3f} s; "
          f"launch {launch}", flush=True)
    sys.stdout.flush()


if __name__ == "__main__":
    main()
