"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

FP64 gate: maximum pointwise relative error of Phi <= 1e-12 (the maximum
relative error measure of Sect. 5; Phi < 0 everywhere for rho >= 0).
"""

import functools
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _yyg():
    from paper_1806_04593_amd import yyg
    return yyg


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu_solve(desc, rho, precision="fp64", grid=None):
    torch = _torch()
    yyg = _yyg()
    g = grid or yyg.Grid(desc, 0)
    if precision != "fp64":
        g.prepare(precision)
    d_rho = torch.from_numpy(rho).to("cuda")
    d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.upload_rho(d_rho)
    g.solve(d_phi, precision)
    torch.cuda.synchronize()
    return g, d_phi.cpu().numpy()


def _oracle_args(desc):
    return (desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"],
            desc["lmax"], desc["G"])


def _moments_to_q(AC, AS):
    L = AC.shape[2] - 1
    out = np.zeros(AC.shape[:2] + ((L + 1) ** 2,))
    for l in range(L + 1):
        out[:, :, l * l] = AC[:, :, l, 0]
        for m in range(1, l + 1):
            out[:, :, l * l + 2 * m - 1] = AC[:, :, l, m]
            out[:, :, l * l + 2 * m] = AS[:, :, l, m]
    return out


def _moment_bound(desc, rho):
    """Rounding bound of the moment dot products: 2 K u sum_a |rho w T CS|
    (K angular cells, u the FP64 unit roundoff), per (patch, shell, column)."""
    th, ph = O.patch_edges(desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"])
    w = O.overlap_weights(th, ph, desc["delta_theta"], desc["delta_phi"])
    T = O.theta_integrals(th, desc["lmax"])
    C, S = O.phi_integrals(ph, desc["lmax"])
    aC, aS = O.moments(np.abs(rho), w, np.abs(T), np.abs(C), np.abs(S))
    K = desc["n_theta"] * desc["n_phi"]
    return 2.0 * K * np.finfo(np.float64).eps / 2 * _moments_to_q(aC, aS)


def _max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def test_small_full_grid_fp64():
    desc = W.describe("small")
    _say(f"small: n_r=32 {desc['n_theta']}x{desc['n_phi']} lmax=8")
    rho = W.density(desc)
    g, phi = _gpu_solve(desc, rho)
    ref = O.solve(*_oracle_args(desc), rho)
    err = _max_rel(phi, ref)
    _say(f"small max rel err {err:.3e}")
    assert err <= TOL_FP64
    # moments of Eqs. (26)-(27)
    th, ph = O.patch_edges(desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"])
    w = O.overlap_weights(th, ph, desc["delta_theta"], desc["delta_phi"])
    AC, AS = O.moments(rho, w, O.theta_integrals(th, desc["lmax"]), *O.phi_integrals(ph, desc["lmax"]))
    A_ref = _moments_to_q(AC, AS)
    A = g.moments()
    assert np.all(np.abs(A - A_ref) <= _moment_bound(desc, rho))
    np.testing.assert_allclose(g.weights(), w, atol=1e-12)


@pytest.mark.parametrize("case", [
    dict(r=np.array([0.0, 1.0]), res=7.0, lmax=0),                    # one shell, monopole only
    dict(r=np.array([0.5, 0.7, 1.3]), res=11.0, lmax=3),              # tiny, r0 > 0
    dict(r=np.linspace(0.0, 2.0, 131), res=9.0, lmax=11),             # M = 260: ragged M tiles
    dict(r=np.geomspace(1.0, 1e3, 70), res=3.0, lmax=17),             # Q = 324, K = 2852: ragged all round
])
def test_ragged_and_degenerate_shapes(case):
    desc = W.make_desc("edge", case["r"], case["res"], case["lmax"], 0.7, 0)
    _say(f"edge case n_r={len(case['r']) - 1} res={case['res']} lmax={case['lmax']}")
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.1, 1.0, (2, len(case["r"]) - 1, desc["n_theta"], desc["n_phi"]))
    _, phi = _gpu_solve(desc, rho)
    ref = O.solve(*_oracle_args(desc), rho)
    assert _max_rel(phi, ref) <= TOL_FP64


N_F64_VARIANTS = 14
N_PHI_DIRECT = 6
N_PHI_FOLD = 8
N_PHI_LEAN = 4   # phi synthesis only
N_X4 = 12        # tiles on the 4x4x4 FP64 MFMA, every phase (last in each phase's range)
N_BOTH = {0: 8, 4: 6}   # then the folded phi transforms with both halves per block
N_STREAM = 16    # phi synthesis: then the streaming kernels (basis panel in LDS, coefficients to registers)
N_STREAM_WIDE = (6,)   # of which these hold panels up to lmax 131, the others up to 67
N_ANA_STREAM = 8   # phi analysis: then the streaming kernels (colatitude-independent basis in LDS)
N_XCOL = 8         # and last the folded tiles with their last output column on the vector units
N_SEP_LP_TILES = 6   # FP32 phi transforms: tiles first, then the FP32 streaming kernels
N_LP_STREAM = {0: 7, 4: 9}


def _n_x4(phase):
    return N_X4 + N_BOTH.get(phase, 0)


def _x4_base(phase):
    if phase in (0, 4):
        return 2 * N_F64_VARIANTS + N_PHI_DIRECT + N_PHI_FOLD + (N_PHI_LEAN if phase == 4 else 0)
    return 2 * N_F64_VARIANTS


@pytest.mark.parametrize("case", [
    dict(r=np.linspace(0.0, 2.0, 131), res=9.0, lmax=11),
    dict(r=np.geomspace(1.0, 1e3, 70), res=3.0, lmax=17),
])
def test_every_tile_variant_and_split(case):
    """Each FP64 tile shape, and split-K factors 1..7 of the analysis, give the
    oracle's potential."""
    desc = W.make_desc("var", case["r"], case["res"], case["lmax"], 1.0, 0)
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.1, 1.0, (2, len(case["r"]) - 1, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = _yyg().Grid(desc, 0)
    for v in range(N_F64_VARIANTS):
        for split in (1, 3, 7):
            _say(f"variant {v} split {split}")
            g.set_config(v, split, (v + split) % N_F64_VARIANTS)
            _, phi = _gpu_solve(desc, rho, grid=g)
            assert _max_rel(phi, ref) <= TOL_FP64, (v, split)


def test_autotune_keeps_parity():
    desc = W.describe("sn_core")
    rho = W.density(desc)
    g = _yyg().Grid(desc, 0)
    g.autotune("fp64")
    _say(f"autotuned: {g.plan_info()}")
    _, phi = _gpu_solve(desc, rho, grid=g)
    rng = np.random.default_rng(1)
    nR = len(desc["r_edges"]) - 1
    s = np.stack([rng.integers(0, 2, 500), rng.integers(0, nR, 500),
                  rng.integers(0, desc["n_theta"], 500), rng.integers(0, desc["n_phi"], 500)], 1)
    ref = O.solve_sampled(*_oracle_args(desc), rho, s)
    assert _max_rel(phi[s[:, 0], s[:, 1], s[:, 2], s[:, 3]], ref) <= TOL_FP64


def _sampled_parity(name, n_samples, seed=0):
    desc = W.describe(name)
    _say(f"{name}: n_r={len(desc['r_edges']) - 1} {desc['n_theta']}x{desc['n_phi']} lmax={desc['lmax']}")
    rho = W.density(desc)
    g, phi = _gpu_solve(desc, rho)
    rng = np.random.default_rng(seed)
    nR = len(desc["r_edges"]) - 1
    s = np.stack([rng.integers(0, 2, n_samples), rng.integers(0, nR, n_samples),
                  rng.integers(0, desc["n_theta"], n_samples), rng.integers(0, desc["n_phi"], n_samples)], 1)
    # always include the first and last shells and the patch corners
    extra = np.array([[p, n, j, k] for p in (0, 1) for n in (0, nR - 1)
                      for j in (0, desc["n_theta"] - 1) for k in (0, desc["n_phi"] - 1)])
    s = np.concatenate([s, extra])
    ref, (AC, AS) = O.solve_sampled(*_oracle_args(desc), rho, s, return_moments=True)
    got = phi[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
    err = _max_rel(got, ref)
    _say(f"{name} sampled max rel err {err:.3e} over {len(s)} cells")
    A_ref = _moments_to_q(AC, AS)
    A = g.moments()
    ratio = float(np.max(np.abs(A - A_ref) / _moment_bound(desc, rho)))
    _say(f"{name} moments: max |dA| / rounding bound = {ratio:.3e}")
    return err, ratio, g, rho, phi


def test_sn_core_fp64():
    err, ratio, *_ = _sampled_parity("sn_core", 3000)
    assert err <= TOL_FP64
    assert ratio <= 1.0


def test_spheroid_fp64():
    err, ratio, *_ = _sampled_parity("spheroid", 2000)
    assert err <= TOL_FP64
    assert ratio <= 1.0


def test_determinism_and_patch_swap():
    torch = _torch()
    desc = W.describe("sn_core")
    rho = W.density(desc)
    g, phi1 = _gpu_solve(desc, rho)
    _, phi2 = _gpu_solve(desc, rho, grid=g)
    assert np.array_equal(phi1, phi2), "FP64 solve is not bitwise repeatable"
    _, phis = _gpu_solve(desc, rho[::-1].copy(), grid=g)
    assert _max_rel(phis, phi1[::-1]) < 1e-14
    del torch


@pytest.mark.parametrize("n_r, lmax", [(1000, 40), (2559, 31)])
def test_paired_radial_scan_against_oracle(n_r, lmax):
    """The column scan with two columns of one degree per block (lmax >= 31:
    at least 1024 columns) against the oracle on a coarse angular grid:
    n_r 1000 (17-shell chunks) and 2559 (the most shells the paired form's
    LDS holds with two patches: 160 KiB; one more takes one column per
    block, as every grid of the other scan tests does)."""
    yyg = _yyg()
    _torch()
    desc = W.make_desc("scan", np.geomspace(1.0, 1e4, n_r + 1), 30.0, lmax, 1.0, 0)
    rng = np.random.default_rng(n_r + lmax)
    rho = rng.uniform(0.1, 1.0, (2, n_r, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    _, sep = _gpu_solve(desc, rho, grid=g)
    err = _max_rel(sep, ref)
    _say(f"paired scan n_r={n_r} lmax={lmax}: separable max rel err {err:.3e}")
    assert err <= TOL_FP64


def test_separable_shell_limit():
    """The separable form's radial scan keeps a column in LDS: 3413 shells
    fill its 160 KiB with two patches and solve against the oracle; one
    more is refused with YYG_ERR_UNSUPPORTED, and the dense form of that
    plan still solves."""
    yyg = _yyg()
    _torch()
    desc = W.make_desc("deep", np.linspace(0.0, 1.0, 3414), 30.0, 2, 1.0, 0)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 1.0, g.shape)
    _, phi = _gpu_solve(desc, rho, grid=g)
    assert _max_rel(phi, O.solve(*_oracle_args(desc), rho)) <= TOL_FP64
    desc = W.make_desc("deep", np.linspace(0.0, 1.0, 3415), 30.0, 2, 1.0, 0)
    g = yyg.Grid(desc, 0)
    with pytest.raises(yyg.YygError) as ei:
        g.set_method("separable")
    assert ei.value.status == -5
    rho = np.ones(g.shape)
    _, phi = _gpu_solve(desc, rho, grid=g)
    assert _max_rel(phi, O.solve(*_oracle_args(desc), rho)) <= TOL_FP64


@pytest.mark.parametrize("n_r", [449, 1000, 1100, 2000, 2600, 3500])
def test_radial_scan_forms_against_oracle(n_r):
    """Every radial-scan instance on a tiny angular grid (30 deg, lmax 4),
    log-spaced shells over four decades, full grid against the oracle:
    dense scans in registers (n_r <= 1024) and in the loop form beyond;
    the separable column scans with 9, 17, 23, 63 and 63-value chunks per
    lane (n_r 449, 1000, 1100, 2000, 2600: the instance nearest above the
    chunk); 3500 shells, past what the column scan's LDS holds with two
    patches (3413), only in the dense form."""
    yyg = _yyg()
    _torch()
    desc = W.make_desc("scan", np.geomspace(1.0, 1e4, n_r + 1), 30.0, 4, 1.0, 0)
    rng = np.random.default_rng(n_r)
    rho = rng.uniform(0.1, 1.0, (2, n_r, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = yyg.Grid(desc, 0)
    _, dense = _gpu_solve(desc, rho, grid=g)
    err = _max_rel(dense, ref)
    _say(f"scan n_r={n_r}: dense max rel err {err:.3e}")
    assert err <= TOL_FP64
    if n_r <= 3413:
        g.set_method("separable")
        _, sep = _gpu_solve(desc, rho, grid=g)
        err = _max_rel(sep, ref)
        _say(f"scan n_r={n_r}: separable max rel err {err:.3e}")
        assert err <= TOL_FP64


def test_host_buffers_and_not_ready():
    yyg = _yyg()
    _torch()
    desc = W.describe("small")
    rho = W.density(desc)
    g = yyg.Grid(desc, 0)
    phi = np.zeros(g.shape)
    with pytest.raises(yyg.YygError) as ei:
        g.solve(phi)
    assert ei.value.status == -4
    g.upload_rho(rho)
    g.solve(phi)
    ref = O.solve(*_oracle_args(desc), rho)
    assert _max_rel(phi, ref) <= TOL_FP64


# ---------------------------------------------------------------------------
# separable form (phi / theta transforms and rotated cross-patch moments)
# ---------------------------------------------------------------------------

def test_separable_small_full_grid():
    desc = W.describe("small")
    rho = W.density(desc)
    g = _yyg().Grid(desc, 0)
    g.set_method("separable")
    _, phi = _gpu_solve(desc, rho, grid=g)
    ref = O.solve(*_oracle_args(desc), rho)
    err = _max_rel(phi, ref)
    _say(f"separable small max rel err {err:.3e}")
    assert err <= TOL_FP64


@pytest.mark.parametrize("case", [
    dict(r=np.array([0.0, 1.0]), res=7.0, lmax=0),
    dict(r=np.array([0.5, 0.7, 1.3]), res=11.0, lmax=3),
    dict(r=np.linspace(0.0, 2.0, 131), res=9.0, lmax=11),
    dict(r=np.geomspace(1.0, 1e3, 70), res=3.0, lmax=17),
])
def test_separable_ragged_shapes(case):
    desc = W.make_desc("edge", case["r"], case["res"], case["lmax"], 0.7, 0)
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.1, 1.0, (2, len(case["r"]) - 1, desc["n_theta"], desc["n_phi"]))
    g = _yyg().Grid(desc, 0)
    g.set_method("separable")
    _, phi = _gpu_solve(desc, rho, grid=g)
    ref = O.solve(*_oracle_args(desc), rho)
    assert _max_rel(phi, ref) <= TOL_FP64
    # the folded LDS-basis phi kernels and the LDS-free folded synthesis on
    # the same shapes (odd and even n_phi, lmax 0: no sin half)
    for f in (0, 4, 7, 8, 11):
        g.sep_config(0, 2 * N_F64_VARIANTS + N_PHI_DIRECT + min(f, N_PHI_FOLD - 1))
        g.sep_config(4, 2 * N_F64_VARIANTS + N_PHI_DIRECT + f)   # f >= 8: the LDS-free synthesis
        _say(f"separable ragged, folded phi variant {f}: {g.sep_info()}")
        _, phi_f = _gpu_solve(desc, rho, grid=g)
        assert _max_rel(phi_f, ref) <= TOL_FP64, f
    # the streaming phi kernels and the extra-column analysis tiles on the
    # same shapes (every one that holds the degree)
    yyg = _yyg()
    n0, n4 = g.sep_variant_count(0), g.sep_variant_count(4)
    ran = 0
    for phase, lo, hi in ((0, n0 - N_XCOL - N_ANA_STREAM, n0), (4, n4 - N_STREAM, n4)):
        for v in range(lo, hi):
            try:
                g.sep_config(phase, v)
            except yyg.YygError as e:
                assert e.status == yyg.ERR_UNSUPPORTED, (phase, v)
                continue
            _, phi_s = _gpu_solve(desc, rho, grid=g)
            err = _max_rel(phi_s, ref)
            _say(f"separable ragged, {g.sep_kernel(phase)}: {err:.2e}")
            assert err <= TOL_FP64, (phase, v, g.sep_kernel(phase), err)
            ran += 1
        g.sep_config(phase, 10)
    assert ran >= N_XCOL + N_ANA_STREAM
    # the separable form keeps its moments column-major; the export is the
    # same [patch][shell][q] array as after a dense solve
    th, ph = O.patch_edges(desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"])
    w = O.overlap_weights(th, ph, desc["delta_theta"], desc["delta_phi"])
    AC, AS = O.moments(rho, w, O.theta_integrals(th, desc["lmax"]), *O.phi_integrals(ph, desc["lmax"]))
    assert np.all(np.abs(g.moments() - _moments_to_q(AC, AS)) <= _moment_bound(desc, rho))
    # last, the FP32 streaming kernels of the separable FP32 solve (the
    # moments it leaves carry FP32 rounding)
    torch = _torch()
    for phase, n in N_LP_STREAM.items():
        for t in range(N_SEP_LP_TILES, N_SEP_LP_TILES + n):
            st = yyg.lib().yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, t)
            if st == yyg.ERR_UNSUPPORTED:
                continue
            assert st == 0, (phase, t, st)
            d_phi = torch.empty(g.shape, dtype=torch.float64, device="cuda")
            g.upload_rho(torch.from_numpy(rho).to("cuda"))
            g.solve(d_phi, "fp32")
            torch.cuda.synchronize()
            err = _max_rel(d_phi.cpu().numpy(), ref)
            _say(f"separable ragged, fp32 {g.sep_lp_kernel('fp32', phase)}: {err:.2e}")
            assert err <= 1e-5, (phase, t, g.sep_lp_kernel("fp32", phase), err)
        assert yyg.lib().yyg_sep_lp_config(g.handle, yyg.PRECISIONS["fp32"], phase, 0) == 0


@pytest.mark.parametrize("name", ["sn_core", "spheroid"])
def test_separable_workloads_and_dense_agreement(name):
    desc = W.describe(name)
    rho = W.density(desc)
    g = _yyg().Grid(desc, 0)
    _, dense = _gpu_solve(desc, rho, grid=g)
    g.set_method("separable")
    if name == "spheroid":
        g.autotune("fp64")     # exercises the separable phases' variant search
    _, sep = _gpu_solve(desc, rho, grid=g)
    _, sep2 = _gpu_solve(desc, rho, grid=g)
    assert np.array_equal(sep, sep2)
    agree = _max_rel(sep, dense)
    rng = np.random.default_rng(3)
    nR = len(desc["r_edges"]) - 1
    s = np.stack([rng.integers(0, 2, 1500), rng.integers(0, nR, 1500),
                  rng.integers(0, desc["n_theta"], 1500), rng.integers(0, desc["n_phi"], 1500)], 1)
    ref = O.solve_sampled(*_oracle_args(desc), rho, s)
    err = _max_rel(sep[s[:, 0], s[:, 1], s[:, 2], s[:, 3]], ref)
    _say(f"separable {name}: max rel err vs oracle {err:.3e}, vs dense (all cells) {agree:.3e}")
    assert err <= TOL_FP64
    assert agree <= TOL_FP64


PHI_DIRECT_CASES = [
    dict(r=np.geomspace(1.0, 50.0, 22), res=3.0, lmax=40),   # 2L+1 = 81: two basis groups; n_phi > 64
    dict(r=np.linspace(0.0, 1.0, 40), res=1.5, lmax=20),     # n_phi > 128: three basis chunks
]


@functools.lru_cache(maxsize=None)
def _phi_direct_case(i):
    case = PHI_DIRECT_CASES[i]
    desc = W.make_desc("edge", case["r"], case["res"], case["lmax"], 0.8, 0)
    rng = np.random.default_rng(14)
    rho = rng.uniform(0.1, 1.0, (2, len(case["r"]) - 1, desc["n_theta"], desc["n_phi"]))
    return desc, rho, O.solve(*_oracle_args(desc), rho)


@pytest.mark.parametrize("ci", range(len(PHI_DIRECT_CASES)))
@pytest.mark.parametrize("phase", [0, 4])
def test_separable_phi_direct_shapes(ci, phase):
    """The LDS-basis phi kernels (unfolded and folded) where the basis spans
    several 64-row groups and the contraction several 64-wide chunks,
    against the oracle."""
    yyg = _yyg()
    desc, rho, ref = _phi_direct_case(ci)
    nR = rho.shape[1]
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    for d in range(N_PHI_DIRECT + N_PHI_FOLD + (N_PHI_LEAN if phase == 4 else 0)):
        g.sep_config(phase, 2 * N_F64_VARIANTS + d)
        _say(f"phi direct phase {phase} variant {d}: n_r={nR} {desc['n_theta']}x{desc['n_phi']} lmax={desc['lmax']}")
        _, phi = _gpu_solve(desc, rho, grid=g)
        err = _max_rel(phi, ref)
        assert err <= TOL_FP64, (phase, d, err)


@pytest.mark.parametrize("phase", [0, 1, 2, 3, 4])
def test_separable_every_phase_variant(phase):
    """Every tile variant of each phase of the separable form (grouped theta
    phases and moment rotation, phi phases as strided batches over the
    colatitudes), on a ragged grid (n_r 37, 9 deg, lmax 11: 74-row problems,
    37-row rotation problems, so every variant's last row tile is partial),
    against the oracle on the full grid."""
    yyg = _yyg()
    desc = W.make_desc("edge", np.geomspace(1.0, 50.0, 38), 9.0, 11, 0.9, 0)
    rng = np.random.default_rng(12)
    rho = rng.uniform(0.1, 1.0, (2, 37, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    # every tile with one and with three stages of loads in flight; the phi
    # phases also every LDS-basis variant, unfolded and folded; every phase
    # the 4x4x4-MFMA tiles
    n_stream = N_STREAM if phase == 4 else N_ANA_STREAM + N_XCOL if phase == 0 else 0
    assert g.sep_variant_count(phase) == _x4_base(phase) + _n_x4(phase) + n_stream
    for v in range(_x4_base(phase) + _n_x4(phase) + n_stream):
        g.sep_config(phase, v)
        _say(f"separable phase {phase} variant {v}: {g.sep_info()}")
        _, phi = _gpu_solve(desc, rho, grid=g)
        err = _max_rel(phi, ref)
        assert err <= TOL_FP64, (phase, v, err)


def test_phi_stream_variants_odd_row_length():
    """The streaming phi transforms on a grid with an odd number of cells
    per row (7 deg: 41, so the middle cell has no mirror and the last pair
    of folded cells is cut), every variant of both, against the oracle."""
    yyg = _yyg()
    desc = W.make_desc("odd", np.geomspace(1.0, 20.0, 12), 7.0, 9, 0.9, 0)
    assert desc["n_phi"] % 2 == 1
    rng = np.random.default_rng(41)
    rho = rng.uniform(0.1, 1.0, (2, 11, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    for phase, n in ((4, N_STREAM), (0, N_ANA_STREAM + N_XCOL)):
        total = g.sep_variant_count(phase)
        for v in range(total - n, total):
            g.sep_config(phase, v)
            _, phi = _gpu_solve(desc, rho, grid=g)
            err = _max_rel(phi, ref)
            _say(f"odd n_phi {desc['n_phi']}: {g.sep_kernel(phase)} {err:.2e}")
            assert err <= TOL_FP64, (phase, v, err)
        g.sep_config(phase, 10)


@pytest.mark.parametrize("case", [
    dict(name="lmax64", res=5.0, lmax=64, nr=5),
    dict(name="lmax32_odd", res=7.0, lmax=32, nr=6),
])
def test_phi_analysis_extra_column_tiles(case):
    """The folded phi-analysis tiles whose last output column is summed on
    the vector units, at degrees where that column is active (lmax 64: L + 1
    = 65 columns in 64-wide tiles, and in 32-wide ones on their second
    tile; lmax 32 on a grid with an odd number of cells per row, 41),
    every variant against the oracle."""
    yyg = _yyg()
    desc = W.make_desc("edge", np.geomspace(1.0, 9.0, case["nr"] + 1), case["res"], case["lmax"], 0.9, 0)
    rng = np.random.default_rng(53)
    rho = rng.uniform(0.1, 1.0, (2, case["nr"], desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    total = g.sep_variant_count(0)
    for v in range(total - N_XCOL, total):
        g.sep_config(0, v)
        _, phi = _gpu_solve(desc, rho, grid=g)
        err = _max_rel(phi, ref)
        _say(f"{case['name']} n_phi {desc['n_phi']}: {g.sep_kernel(0)} {err:.2e}")
        assert err <= TOL_FP64, (v, err)


def test_phi_stream_variants_at_high_degree():
    """The streaming phi synthesis at lmax 80 (21 steps of four cosine and
    four sine columns): the variants whose LDS panel holds only lmax <= 67
    are refused with YYG_ERR_UNSUPPORTED, the wide-panel variant matches
    the oracle on a ragged grid (n_r 5, 5 deg).  (The oracle's unnormalised
    associated Legendre values leave FP64's range near lmax 90.)"""
    yyg = _yyg()
    desc = W.make_desc("edge", np.geomspace(1.0, 9.0, 6), 5.0, 80, 0.9, 0)
    rng = np.random.default_rng(31)
    rho = rng.uniform(0.1, 1.0, (2, 5, desc["n_theta"], desc["n_phi"]))
    ref = O.solve(*_oracle_args(desc), rho)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    base = _x4_base(4) + _n_x4(4)
    for u in range(N_STREAM):
        if u in N_STREAM_WIDE:
            continue
        with pytest.raises(yyg.YygError) as ei:
            g.sep_config(4, base + u)
        assert ei.value.status == yyg.ERR_UNSUPPORTED
    for u in N_STREAM_WIDE:
        g.sep_config(4, base + u)
        _say(f"phi stream at lmax 80: {g.sep_kernel(4)}")
        _, phi = _gpu_solve(desc, rho, grid=g)
        err = _max_rel(phi, ref)
        assert err <= TOL_FP64, err


def test_separable_phase_alone():
    """yyg_sep_phase: one phase launched alone after a solve recomputes that
    phase's output from what the solve left (the phi synthesis rewrites the
    potential bit for bit); without the separable form it is not ready."""
    torch = _torch()
    yyg = _yyg()
    desc = W.describe("small")
    rho = W.density(desc)
    g = yyg.Grid(desc, 0)
    d_rho = torch.from_numpy(rho).to("cuda")
    d_phi = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    g.upload_rho(d_rho)
    with pytest.raises(yyg.YygError) as ei:
        g.sep_phase(4, d_phi)
    assert ei.value.status == -4          # YYG_ERR_NOT_READY: dense method
    g.set_method("separable")
    # the default tiles, then the streaming phi synthesis and analysis
    for streaming in (False, True):
        if streaming:
            g.sep_config(0, g.sep_variant_count(0) - N_XCOL - N_ANA_STREAM)
            g.sep_config(4, g.sep_variant_count(4) - N_STREAM)
        g.solve(d_phi)
        torch.cuda.synchronize()
        ref = d_phi.clone()
        for phase in range(5):
            d_phi.fill_(0.0)
            for _ in range(2):
                g.sep_phase(phase, d_phi)
            if phase < 4:
                g.sep_phase(4, d_phi)
            torch.cuda.synchronize()
            assert torch.equal(d_phi, ref), (streaming, phase)


@pytest.mark.parametrize("method", ["dense", "separable", "separable_streaming"])
def test_solve_captures_in_a_graph(method):
    """A solve on device buffers is asynchronous and allocation-free, so it
    records into a HIP graph: replays (with eager work and synchronisations
    between them) reproduce the eager result bit for bit."""
    torch = _torch()
    yyg = _yyg()
    desc = W.describe("small")
    rho = W.density(desc)
    g = yyg.Grid(desc, 0)
    if method != "dense":
        g.set_method("separable")
    if method == "separable_streaming":
        # the streaming phi synthesis and analysis (persistent grids)
        g.sep_config(0, g.sep_variant_count(0) - N_XCOL - N_ANA_STREAM)
        g.sep_config(4, g.sep_variant_count(4) - N_STREAM)
    d_rho = torch.from_numpy(rho).to("cuda")
    d_phi = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    g.upload_rho(d_rho)
    g.solve(d_phi)
    torch.cuda.synchronize()
    eager = d_phi.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.solve(d_phi)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.solve(d_phi)
    for rep in range(3):
        d_phi.fill_(0.0)
        _ = (torch.arange(4096, device="cuda", dtype=torch.float64) * rep).sum().item()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(d_phi, eager), (method, rep)
    assert _max_rel(eager.cpu().numpy(), O.solve(*_oracle_args(desc), rho)) <= TOL_FP64
