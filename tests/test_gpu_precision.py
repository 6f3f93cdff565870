"""Reduced-precision angular contractions (FP32, BF16 x 3, FP16 x 2) against
the FP64 oracle.  Gates (maximum pointwise relative error of Phi):
split BF16 x 3 and FP16 x 2 <= 1e-6; FP32 <= 1e-4 (its error is reported).
"""

import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16x3": 1e-6, "fp16x2": 1e-6}
N_LP_VARIANTS = 5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle_args(desc):
    return (desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"],
            desc["lmax"], desc["G"])


def _solve(g, rho, precision):
    torch = _torch()
    d_rho = torch.from_numpy(rho).to("cuda")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.upload_rho(d_rho)
    g.solve(d_phi, precision)
    torch.cuda.synchronize()
    return d_phi.cpu().numpy()


def _grid(desc):
    from paper_1806_04593_amd import yyg
    return yyg.Grid(desc, 0)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x2"])
def test_small_full_grid(precision):
    desc = W.describe("small")
    rho = W.density(desc)
    g = _grid(desc)
    g.prepare(precision)
    phi = _solve(g, rho, precision)
    ref = O.solve(*_oracle_args(desc), rho)
    err = float(np.max(np.abs(phi - ref) / np.abs(ref)))
    _say(f"small {precision}: max rel err {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x2"])
def test_every_variant_ragged(precision):
    desc = W.make_desc("var", np.geomspace(1.0, 1e3, 70), 3.0, 17, 1.0, 0)
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.1, 1.0, (2, 69, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = _grid(desc)
    g.prepare(precision)
    for v in range(N_LP_VARIANTS):
        for split in (1, 5):
            g.set_config(v, split, (v + 1) % N_LP_VARIANTS, precision)
            phi = _solve(g, rho, precision)
            err = float(np.max(np.abs(phi - ref) / np.abs(ref)))
            _say(f"{precision} variant {v} split {split}: {err:.3e}")
            assert err <= TOL[precision], (v, split)


@pytest.mark.parametrize("name", ["sn_core", "spheroid"])
def test_workload_errors(name):
    desc = W.describe(name)
    rho = W.density(desc)
    nR = len(desc["r_edges"]) - 1
    rng = np.random.default_rng(2)
    s = np.stack([rng.integers(0, 2, 1500), rng.integers(0, nR, 1500),
                  rng.integers(0, desc["n_theta"], 1500), rng.integers(0, desc["n_phi"], 1500)], 1)
    ref = O.solve_sampled(*_oracle_args(desc), rho, s)
    g = _grid(desc)
    errs = {}
    for precision in ("fp32", "bf16x3", "fp16x2"):
        g.prepare(precision)
        g.autotune(precision)
        phi = _solve(g, rho, precision)
        got = phi[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
        errs[precision] = float(np.max(np.abs(got - ref) / np.abs(ref)))
        _say(f"{name} {precision}: max rel err {errs[precision]:.3e} ({g.plan_info(precision)})")
    for precision, err in errs.items():
        assert err <= TOL[precision], (precision, err)


# ---------------------------------------------------------------------------
# the separable form's phi transforms in FP32 and BF16 x 3 (theta transforms,
# rotation and radial sums in FP64)
# ---------------------------------------------------------------------------

N_SEP_LP_TILES = 6
N_STREAM32 = 9   # FP32 phi synthesis: the FP32 streaming kernels after the tiles
N_ANA_STREAM32 = 7   # FP32 phi analysis: the FP32 streaming kernels after the tiles


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_separable_reduced_precision_every_tile(precision):
    """Every reduced-precision tile of both phi transforms on a ragged grid
    (n_r 37, 9 deg, lmax 11) and the small workload, full grid against the
    oracle; autotuned tiles on sn_core sampled."""
    torch = _torch()
    desc = W.make_desc("edge", np.geomspace(1.0, 50.0, 38), 9.0, 11, 0.9, 0)
    rng = np.random.default_rng(31)
    rho = rng.uniform(0.1, 1.0, (2, 37, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = _grid(desc)
    g.set_method("separable")
    for phase in (0, 4):
        n = N_SEP_LP_TILES + ((N_STREAM32 if phase == 4 else N_ANA_STREAM32) if precision == "fp32" else 0)
        for t in range(n):
            _set_lp_tile(g, precision, phase, t)
            phi = _solve(g, rho, precision)
            err = float(np.max(np.abs(phi - ref) / np.abs(ref)))
            _say(f"separable {precision} phase {phase} tile {t} ({g.sep_lp_kernel(precision, phase)}): {err:.3e}")
            assert err <= TOL[precision], (phase, t, err)
    for name in ("small", "sn_core"):
        desc = W.describe(name)
        rho = W.density(desc)
        g = _grid(desc)
        g.set_method("separable")
        d_rho = torch.from_numpy(rho).to("cuda")
        g.upload_rho(d_rho)
        g.autotune(precision)
        phi = _solve(g, rho, precision)
        if name == "small":
            ref = O.solve(*_oracle_args(desc), rho)
            err = float(np.max(np.abs(phi - ref) / np.abs(ref)))
        else:
            s = np.stack([rng.integers(0, 2, 800), rng.integers(0, 400, 800), rng.integers(0, desc["n_theta"], 800),
                          rng.integers(0, desc["n_phi"], 800)], 1)
            ref = O.solve_sampled(*_oracle_args(desc), rho, s)
            got = phi[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
            err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        _say(f"separable {precision} {name}: {err:.3e}")
        assert err <= TOL[precision], (name, err)


def test_separable_stream32_only_for_the_fp32_synthesis():
    """The FP32 streaming kernels are choices of the FP32 phi transforms
    only: BF16 x 3 refuses them, and each transform has its own count."""
    from paper_1806_04593_amd import yyg
    desc = W.make_desc("edge", np.geomspace(1.0, 50.0, 38), 9.0, 11, 0.9, 0)
    g = _grid(desc)
    g.set_method("separable")
    L = yyg.lib()
    assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], 4, N_SEP_LP_TILES) == 0
    assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], 0, N_SEP_LP_TILES) == 0
    assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["bf16x3"], 4, N_SEP_LP_TILES) == yyg.ERR_UNSUPPORTED
    assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["bf16x3"], 0, N_SEP_LP_TILES) == yyg.ERR_UNSUPPORTED
    # past a transform's own kernels: refused, and past every tile index a
    # precision has, an invalid argument
    n_max = N_SEP_LP_TILES + max(N_STREAM32, N_ANA_STREAM32)
    for phase, n in ((4, N_STREAM32), (0, N_ANA_STREAM32)):
        assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, N_SEP_LP_TILES + n - 1) == 0
        for t in range(N_SEP_LP_TILES + n, n_max):
            assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, t) == yyg.ERR_UNSUPPORTED
        assert L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, n_max) == yyg.ERR_INVALID_ARG


def test_separable_fp32_streams_odd_row_length():
    """The FP32 streaming phi kernels on a grid with an odd number of cells
    per row (7 deg: 41; the middle cell has no mirror), every analysis and
    synthesis variant, full grid against the oracle."""
    _torch()
    desc = W.make_desc("odd", np.geomspace(1.0, 20.0, 12), 7.0, 9, 0.9, 0)
    assert desc["n_phi"] % 2 == 1
    rng = np.random.default_rng(43)
    rho = rng.uniform(0.1, 1.0, (2, 11, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = _grid(desc)
    g.set_method("separable")
    for phase, n in ((0, N_ANA_STREAM32), (4, N_STREAM32)):
        for t in range(N_SEP_LP_TILES, N_SEP_LP_TILES + n):
            _set_lp_tile(g, "fp32", phase, t)
            phi = _solve(g, rho, "fp32")
            err = float(np.max(np.abs(phi - ref) / np.abs(ref)))
            _say(f"odd n_phi {desc['n_phi']}: fp32 phase {phase} {g.sep_lp_kernel('fp32', phase)} {err:.2e}")
            assert err <= 1e-6, (phase, t, err)
        _set_lp_tile(g, "fp32", phase, 0)


def test_separable_fp32_streams_at_high_degree():
    """The FP32 streaming phi kernels at lmax 80 on a ragged grid (n_r 5,
    5 deg): the synthesis kernels whose LDS panel holds only lmax <= 67 are
    refused with YYG_ERR_UNSUPPORTED; the two wide-panel ones (the fifth and
    seventh) and every analysis kernel (bounded by the row length, not the
    degree) match the oracle."""
    from paper_1806_04593_amd import yyg
    _torch()
    desc = W.make_desc("edge", np.geomspace(1.0, 9.0, 6), 5.0, 80, 0.9, 0)
    rng = np.random.default_rng(37)
    rho = rng.uniform(0.1, 1.0, (2, 5, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = _grid(desc)
    g.set_method("separable")
    L = yyg.lib()
    wide = (4, 6)
    for phase, n in ((4, N_STREAM32), (0, N_ANA_STREAM32)):
        for v in range(n):
            st = L.yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, N_SEP_LP_TILES + v)
            if phase == 4 and v not in wide:
                assert st == yyg.ERR_UNSUPPORTED, (phase, v, st)
                continue
            assert st == 0, (phase, v, st)
            phi = _solve(g, rho, "fp32")
            err = float(np.max(np.abs(phi - ref) / np.abs(ref)))
            _say(f"lmax 80: fp32 phase {phase} {g.sep_lp_kernel('fp32', phase)} {err:.2e}")
            assert err <= TOL["fp32"], (phase, v, err)
        _set_lp_tile(g, "fp32", phase, 0)


def _set_lp_tile(g, precision, phase, t):
    """Reduced-precision tile t of phi phase `phase` (yyg_sep_lp_config)."""
    from paper_1806_04593_amd import yyg
    assert yyg.lib().yyg_sep_lp_config(g.handle, yyg.PRECISIONS[precision], int(phase), int(t)) == 0


def test_separable_fp16x2_refused():
    from paper_1806_04593_amd import yyg
    _torch()
    desc = W.describe("small")
    g = _grid(desc)
    g.set_method("separable")
    rho = W.density(desc)
    with pytest.raises(yyg.YygError) as ei:
        _solve(g, rho, "fp16x2")
    assert ei.value.status == -5
