"""GPU parity at the largest single-GPU workload and at the uneven 64-field
batch, in the launch configuration the benchmark times.

binary: n_r = 1000 log-spaced shells on [1e5, 1e10] cm, 0.5 deg Yin-Yang
(182 x 542 cells per patch), lmax = 64, 1.97e8 cells.  The oracle computes
the moments and radial sums in full and the synthesis at sampled outputs
(2000 random cells plus the patch corners on the first, last and a middle
shell, plus random cells of the first and last shells).  Gate: the maximum
relative error of Sect. 5 over the samples, <= 1e-12 for FP64, the split
precisions <= 1e-6, FP32 <= 1e-4; the moments within the FP64 rounding
bound of their dot products.

batch64: the 64 uneven fields of the batched workload (n_r in [100, 600],
2, 3 or 4 deg, lmax in [10, 30], seeded as the benchmark seeds them),
solved in one batched launch sequence and checked on 8 fields.
"""

import functools
import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4, "bf16x3": 1e-6, "fp16x2": 1e-6}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _yyg():
    from paper_1806_04593_amd import yyg
    return yyg


def _max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _samples(desc, k, seed):
    nR, nt, np_ = len(desc["r_edges"]) - 1, desc["n_theta"], desc["n_phi"]
    rng = np.random.default_rng(seed)
    s = [np.stack([rng.integers(0, 2, k), rng.integers(0, nR, k), rng.integers(0, nt, k),
                   rng.integers(0, np_, k)], 1)]
    corners = [(p, n, j, kk) for p in (0, 1) for n in (0, nR // 2, nR - 1) for j in (0, nt - 1)
               for kk in (0, np_ - 1)]
    s.append(np.array(corners))
    for n in (0, nR - 1):   # first and last shells
        s.append(np.stack([rng.integers(0, 2, 100), np.full(100, n), rng.integers(0, nt, 100),
                           rng.integers(0, np_, 100)], 1))
    return np.concatenate(s)


@functools.lru_cache(maxsize=None)
def _binary():
    """Workload, density, samples, the oracle at the samples and its moments."""
    desc = W.describe("binary")
    rho = W.density(desc)
    s = _samples(desc, 2000, 55)
    _say(f"binary: oracle at {len(s)} samples (moments and radial sums in full)")
    ref, (AC, AS) = O.solve_sampled(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"],
                                    desc["delta_phi"], desc["lmax"], desc["G"], rho, s, return_moments=True)
    return desc, rho, s, ref, AC, AS


@functools.lru_cache(maxsize=None)
def _binary_grid():
    torch = _torch()
    desc, rho, *_ = _binary()
    g = _yyg().Grid(desc, 0)
    d_rho = torch.from_numpy(rho).to("cuda")
    g.upload_rho(d_rho)
    return g, d_rho


def _solve(g, precision="fp64"):
    torch = _torch()
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.solve(d_phi, precision)
    torch.cuda.synchronize()
    return d_phi


def _at(d_phi, s):
    import torch
    idx = torch.from_numpy(s).to(d_phi.device)
    return d_phi[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]].cpu().numpy()


def _moments_to_q(AC, AS):
    L = AC.shape[2] - 1
    out = np.zeros(AC.shape[:2] + ((L + 1) ** 2,))
    for l in range(L + 1):
        out[:, :, l * l] = AC[:, :, l, 0]
        for m in range(1, l + 1):
            out[:, :, l * l + 2 * m - 1] = AC[:, :, l, m]
            out[:, :, l * l + 2 * m] = AS[:, :, l, m]
    return out


def test_binary_separable_fp64():
    """The benchmark's headline path: separable FP64, autotuned as the
    benchmark does; Phi at the samples and the exported moments."""
    desc, rho, s, ref, AC, AS = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    g.autotune("fp64")
    _say(f"binary separable: variants {g.sep_info()} phi kernels {g.sep_kernel(0)} / {g.sep_kernel(4)}")
    d_phi = _solve(g)
    err = _max_rel(_at(d_phi, s), ref)
    _say(f"binary separable FP64: max rel err {err:.3e} over {len(s)} samples")
    assert err <= TOL["fp64"]
    # the moments of Eqs. (26)-(27) within the rounding bound of their dot
    # products, 2 K u sum |rho w T CS| (K angular cells)
    th, ph = O.patch_edges(desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"])
    w = O.overlap_weights(th, ph, desc["delta_theta"], desc["delta_phi"])
    T = O.theta_integrals(th, desc["lmax"])
    C, S = O.phi_integrals(ph, desc["lmax"])
    aC, aS = O.moments(np.abs(rho), w, np.abs(T), np.abs(C), np.abs(S))
    K = desc["n_theta"] * desc["n_phi"]
    bound = 2.0 * K * np.finfo(np.float64).eps / 2 * _moments_to_q(aC, aS)
    got = g.moments()
    assert np.all(np.abs(got - _moments_to_q(AC, AS)) <= bound)
    g.set_method("dense")


def test_binary_dense_fp64():
    desc, rho, s, ref, *_ = _binary()
    g, _ = _binary_grid()
    g.set_method("dense")
    d_phi = _solve(g)
    err = _max_rel(_at(d_phi, s), ref)
    _say(f"binary dense FP64 {g.plan_info('fp64')}: max rel err {err:.3e}")
    assert err <= TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x2"])
def test_binary_dense_reduced_precision(precision):
    desc, rho, s, ref, *_ = _binary()
    g, _ = _binary_grid()
    g.set_method("dense")
    g.prepare(precision)
    d_phi = _solve(g, precision)
    err = _max_rel(_at(d_phi, s), ref)
    _say(f"binary dense {precision}: max rel err {err:.3e}")
    assert err <= TOL[precision]


@functools.lru_cache(maxsize=None)
def _batch64():
    descs = W.batch_descs(64)
    rhos = [W.density(d) for d in descs]
    return descs, rhos


@pytest.mark.parametrize("precision", ["fp64", "fp16x2", "fp64-separable"])
def test_batch64_full_sizes(precision):
    """All 64 fields in one batched solve (dense FP64, dense FP16x2, and the
    separable form's grouped phases); 8 fields (the largest and the smallest
    among them) checked against the oracle at 300 samples each."""
    torch = _torch()
    yyg = _yyg()
    descs, rhos = _batch64()
    grids = [yyg.Grid(d, 0) for d in descs]
    sep = precision == "fp64-separable"
    if sep:
        precision = "fp64"
        for g in grids:
            g.set_method("separable")
    if precision != "fp64":
        for g in grids:
            g.prepare(precision)
    d_rho = [torch.from_numpy(r).to("cuda") for r in rhos]
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]
    b = yyg.Batch(grids, precision)
    assert (b.info()["var_theta_ana"] >= 0) == sep
    stream = torch.cuda.Stream()
    b.solve(d_rho, d_phi, stream=stream)
    b.solve(d_rho, d_phi, stream=stream)   # a graph replay
    stream.synchronize()
    sizes = np.array([len(d["r_edges"]) - 1 for d in descs]) * np.array([d["n_theta"] * d["n_phi"] for d in descs])
    order = np.argsort(sizes)
    check = sorted(set(order[:3].tolist() + order[-3:].tolist() + [21, 42]))
    worst = 0.0
    for f in check:
        d = descs[f]
        s = _samples(d, 300, 100 + f)
        ref = O.solve_sampled(d["r_edges"], d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"],
                              d["lmax"], d["G"], rhos[f], s)
        err = _max_rel(_at(d_phi[f], s), ref)
        _say(f"batch64 {precision} field {f} (n_r {len(d['r_edges']) - 1}, {d['n_theta']}x{d['n_phi']}, "
             f"lmax {d['lmax']}): {err:.3e}")
        worst = max(worst, err)
    b.close()
    assert worst <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_binary_separable_reduced_precision(precision):
    """The separable form with its phi transforms in FP32 / BF16 x 3,
    autotuned as the benchmark runs it, at the binary workload's samples."""
    desc, rho, s, ref, *_ = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    g.autotune(precision)
    d_phi = _solve(g, precision)
    err = _max_rel(_at(d_phi, s), ref)
    _say(f"binary separable {precision} ({g.sep_lp_kernel(precision, 0)} / {g.sep_lp_kernel(precision, 4)}): "
         f"max rel err {err:.3e}")
    assert err <= TOL[precision]
    g.set_method("dense")


N_STREAM = 16         # streaming phi-synthesis variants, last in the phase's range (all hold lmax 64)


def test_binary_separable_stream_variants():
    """Each streaming phi-synthesis variant at the binary workload (the
    other phases as the autotuner left them), at the oracle's samples."""
    desc, rho, s, ref, *_ = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    n = g.sep_variant_count(4)
    for v in range(n - N_STREAM, n):
        g.sep_config(4, v)
        d_phi = _solve(g)
        err = _max_rel(_at(d_phi, s), ref)
        _say(f"binary separable, phi synthesis {g.sep_kernel(4)}: max rel err {err:.3e}")
        assert err <= TOL["fp64"]
    g.set_method("dense")


N_STREAM32_L64 = 9   # FP32 streaming phi-synthesis kernels (tiles 6 onwards), all holding lmax 64


def test_binary_separable_fp32_stream_variants():
    """Each FP32 streaming phi-synthesis kernel that holds lmax 64 at the
    binary workload's samples (the FP32 analysis tile as the autotuner
    left it)."""
    from paper_1806_04593_amd import yyg
    desc, rho, s, ref, *_ = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    for t in range(6, 6 + N_STREAM32_L64):
        assert yyg.lib().yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], 4, t) == 0
        d_phi = _solve(g, "fp32")
        err = _max_rel(_at(d_phi, s), ref)
        _say(f"binary separable fp32, phi synthesis {g.sep_lp_kernel('fp32', 4)}: max rel err {err:.3e}")
        assert err <= TOL["fp32"] and err <= 1e-6
    g.set_method("dense")


N_ANA_STREAM = 8   # streaming phi-analysis variants (all hold h = 271), before the N_XCOL last ones
N_XCOL = 8         # folded analysis tiles with the last output column on the vector units, last in the range


def test_binary_separable_analysis_stream_variants():
    """Each streaming phi-analysis variant at the binary workload's samples
    (weights applied to the density pairs as they load), and the moments
    they lead to within the FP64 rounding bound."""
    desc, rho, s, ref, AC, AS = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    n = g.sep_variant_count(0) - N_XCOL
    for v in range(n - N_ANA_STREAM, n):
        g.sep_config(0, v)
        d_phi = _solve(g)
        err = _max_rel(_at(d_phi, s), ref)
        _say(f"binary separable, phi analysis {g.sep_kernel(0)}: max rel err {err:.3e}")
        assert err <= TOL["fp64"]
    g.set_method("dense")


def test_binary_separable_analysis_extra_column_tiles():
    """Each folded phi-analysis tile whose last output column (cos 64, the
    65th of the even half) is summed on the vector units, at the binary
    workload's samples."""
    desc, rho, s, ref, AC, AS = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    n = g.sep_variant_count(0)
    for v in range(n - N_XCOL, n):
        g.sep_config(0, v)
        d_phi = _solve(g)
        err = _max_rel(_at(d_phi, s), ref)
        _say(f"binary separable, phi analysis {g.sep_kernel(0)}: max rel err {err:.3e}")
        assert err <= TOL["fp64"]
    g.set_method("dense")


N_ANA_STREAM32 = 7   # FP32 streaming phi-analysis kernels (tiles 6 onwards of the FP32 analysis)


def test_binary_separable_fp32_analysis_stream_variants():
    """Each FP32 streaming phi-analysis kernel at the binary workload's
    samples (the FP32 synthesis as the autotuner left it)."""
    from paper_1806_04593_amd import yyg
    desc, rho, s, ref, *_ = _binary()
    g, _ = _binary_grid()
    g.set_method("separable")
    for t in range(6, 6 + N_ANA_STREAM32):
        assert yyg.lib().yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], 0, t) == 0
        d_phi = _solve(g, "fp32")
        err = _max_rel(_at(d_phi, s), ref)
        _say(f"binary separable fp32, phi analysis {g.sep_lp_kernel('fp32', 0)}: max rel err {err:.3e}")
        assert err <= 1e-6
    g.set_method("dense")
