"""GPU parity of the full-sphere polar-grid mode (one patch, unit weights,
no patch combination; the method of Sect. 2) against the oracle's polar
solve, through the C ABI, for both solution methods and every precision."""

import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4, "bf16x3": 1e-6, "fp16x2": 1e-6}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _solve(desc, rho, method="dense", precision="fp64", autotune=False):
    torch = _torch()
    from paper_1806_04593_amd import yyg
    g = yyg.Grid(desc, 0)
    assert g.shape == (1, len(desc["r_edges"]) - 1, desc["n_theta"], desc["n_phi"])
    if precision != "fp64":
        g.prepare(precision)
    if method != "dense":
        g.set_method(method)
    d_rho = torch.from_numpy(rho).to("cuda")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.upload_rho(d_rho)
    if autotune:
        g.autotune(precision)
    g.solve(d_phi, precision)
    torch.cuda.synchronize()
    return g, d_phi.cpu().numpy()


def _oracle(desc, rho):
    return O.solve_polar(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["lmax"], desc["G"], rho)


def _max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


@pytest.mark.parametrize("method", ["dense", "separable"])
def test_polar_small_full_grid_fp64(method):
    desc = W.describe("polar_small")
    rho = W.density(desc)
    _say(f"polar_small {method}: n_r=32 36x72 lmax=8")
    g, phi = _solve(desc, rho, method)
    err = _max_rel(phi, _oracle(desc, rho))
    _say(f"polar_small {method} max rel err {err:.3e}")
    assert err <= TOL["fp64"]
    np.testing.assert_array_equal(g.weights(), np.ones((36, 72)))
    assert g.moments().shape == (1, 32, 81)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x2"])
def test_polar_small_reduced_precision(precision):
    desc = W.describe("polar_small")
    rho = W.density(desc)
    _say(f"polar_small {precision}")
    _, phi = _solve(desc, rho, "dense", precision)
    err = _max_rel(phi, _oracle(desc, rho))
    _say(f"polar_small {precision} max rel err {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("method", ["dense", "separable"])
@pytest.mark.parametrize("case", [
    dict(r=np.array([0.0, 1.0]), nt=5, np_=9, lmax=0),
    dict(r=np.linspace(0.0, 2.0, 131), nt=25, np_=51, lmax=13),      # ragged tiles in every dimension
    dict(r=np.geomspace(1.0, 1e3, 70), nt=61, np_=119, lmax=30),
])
def test_polar_ragged_shapes(method, case):
    desc = W.make_polar_desc("edge", case["r"], 10.0, case["lmax"], 0.7, 0)
    desc.update(n_theta=case["nt"], n_phi=case["np_"])
    _say(f"polar edge {method} n_r={len(case['r']) - 1} {case['nt']}x{case['np_']} lmax={case['lmax']}")
    rng = np.random.default_rng(21)
    rho = rng.uniform(0.1, 1.0, (1, len(case["r"]) - 1, case["nt"], case["np_"]))
    _, phi = _solve(desc, rho, method)
    assert _max_rel(phi, _oracle(desc, rho)) <= TOL["fp64"]


N_STREAM, N_ANA_STREAM, N_XCOL = 16, 8, 8   # last variants of the phi synthesis / analysis ranges
N_SEP_LP_TILES, N_LP_STREAM = 6, {0: 7, 4: 9}   # FP32 phi transforms: tiles, then streaming kernels


def test_polar_streaming_phi_kernels():
    """The streaming phi kernels on a polar grid (one patch of full rows, 51
    cells: the middle cell has no mirror; n_r 130, lmax 13): every FP64
    streaming synthesis and analysis variant and every extra-column analysis
    tile, then every FP32 streaming kernel of the separable FP32 solve,
    full grid against the oracle's polar solve."""
    torch = _torch()
    from paper_1806_04593_amd import yyg
    desc = W.make_polar_desc("edge", np.linspace(0.0, 2.0, 131), 10.0, 13, 0.7, 0)
    desc.update(n_theta=25, n_phi=51)
    rng = np.random.default_rng(23)
    rho = rng.uniform(0.1, 1.0, (1, 130, 25, 51))
    ref = _oracle(desc, rho)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    d_rho = torch.from_numpy(rho).to("cuda")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda")

    def run(precision):
        g.upload_rho(d_rho)
        g.solve(d_phi, precision)
        torch.cuda.synchronize()
        return _max_rel(d_phi.cpu().numpy(), ref)

    for phase, n in ((4, N_STREAM), (0, N_ANA_STREAM + N_XCOL)):
        total = g.sep_variant_count(phase)
        for v in range(total - n, total):
            g.sep_config(phase, v)   # all hold lmax 13 and 26 folded points
            err = run("fp64")
            _say(f"polar {g.sep_kernel(phase)}: {err:.2e}")
            assert err <= TOL["fp64"], (phase, v, err)
        g.sep_config(phase, 10)
    L = yyg.lib()
    for phase, n in N_LP_STREAM.items():
        for t in range(N_SEP_LP_TILES, N_SEP_LP_TILES + n):
            assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, t) == 0, (phase, t)
            err = run("fp32")
            _say(f"polar fp32 {g.sep_lp_kernel('fp32', phase)}: {err:.2e}")
            assert err <= 1e-6, (phase, t, err)
        assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, 0) == 0


@pytest.mark.parametrize("method", ["dense", "separable"])
def test_polar_spherical_symmetry_exact(method):
    """Spherically symmetric density at lmax 25: the shell theorem holds to
    rounding on the polar grid, at every cell (the l > 0 moments vanish)."""
    r = np.geomspace(1e5, 1e9, 201)
    nR = len(r) - 1
    desc = W.make_polar_desc("sym", r, 2.0, 25, W.G_CGS, 0)
    rr = W.rho0(0.5 * (r[:-1] + r[1:]))
    rho = np.broadcast_to(rr[None, :, None, None], (1, nR, desc["n_theta"], desc["n_phi"])).copy()
    _say(f"polar symmetric {method}: n_r=200 90x180 lmax=25")
    _, phi = _solve(desc, rho, method)
    ex = np.array([-(4 * math.pi / (3 * r[n])) * np.sum(rr[:n] * (r[1:n + 1] ** 3 - r[:n] ** 3))
                   - 2 * math.pi * np.sum(rr[n:] * (r[n + 1:] ** 2 - r[n:-1] ** 2)) for n in range(1, nR + 1)])
    ex *= W.G_CGS
    err = float(np.max(np.abs(phi[0] - ex[:, None, None]) / np.abs(ex)[:, None, None]))
    _say(f"polar symmetric {method} max rel err vs shell theorem {err:.3e}")
    assert err < 1e-13


@pytest.mark.parametrize("method", ["dense", "separable"])
def test_polar_sn_core_sampled(method):
    """The sn_core recipe on the 2-degree polar grid (n_r 400, 90 x 180,
    lmax 25), autotuned as the bench runs it; sampled cells against the
    oracle (moments and radial sums in full)."""
    desc = W.describe("polar_sn_core")
    rho = W.density(desc)
    _say(f"polar_sn_core {method}: n_r=400 90x180 lmax=25")
    _, phi = _solve(desc, rho, method, autotune=True)
    rng = np.random.default_rng(31)
    s = np.stack([np.zeros(200, int), rng.integers(0, 400, 200), rng.integers(0, 90, 200),
                  rng.integers(0, 180, 200)], 1)
    ref = O.solve_polar_sampled(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["lmax"], desc["G"], rho, s)
    got = phi[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
    err = _max_rel(got, ref)
    _say(f"polar_sn_core {method} sampled max rel err {err:.3e}")
    assert err <= TOL["fp64"]


def test_batch_mixing_polar_and_yinyang():
    """A batch of polar and Yin-Yang plans equals their single solves."""
    torch = _torch()
    from paper_1806_04593_amd import yyg
    descs = [W.make_polar_desc("p0", np.linspace(0.0, 1.0, 41), 5.0, 12, 1.0, 1000, recipe="small"),
             W.make_desc("y0", np.linspace(0.0, 1.0, 57), 4.0, 10, 1.0, 1001, recipe="small"),
             W.make_polar_desc("p1", np.linspace(0.0, 1.0, 23), 3.0, 20, 1.0, 1002, recipe="small")]
    rhos = [W.density(d) for d in descs]
    grids = [yyg.Grid(d, 0) for d in descs]
    single = []
    for g, r in zip(grids, rhos):
        d_r = torch.from_numpy(r).to("cuda")
        d_p = torch.empty(g.shape, dtype=torch.float64, device="cuda")
        g.upload_rho(d_r)
        g.solve(d_p)
        torch.cuda.synchronize()
        single.append(d_p.cpu().numpy())
    b = yyg.Batch(grids, "fp64")
    d_rho = [torch.from_numpy(r).to("cuda") for r in rhos]
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]
    for rep in range(2):
        for p in d_phi:
            p.zero_()
        torch.cuda.synchronize()
        b.solve(d_rho, d_phi)
        torch.cuda.synchronize()
        for p, ref in zip(d_phi, single):
            assert _max_rel(p.cpu().numpy(), ref) < 1e-13, rep
    # and the polar fields against the oracle
    for i in (0, 2):
        assert _max_rel(d_phi[i].cpu().numpy(), _oracle(descs[i], rhos[i])) <= TOL["fp64"]
