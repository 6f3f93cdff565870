"""CPU tests of the C library's host logic: exported symbols, argument
validation and the FP64 plan tables against the oracle.  No GPU calls."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W
from paper_1806_04593_amd import yyg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "yyg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(yyg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = yyg.lib()
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(yyg.EXPORTS) == names


def test_single_hip_runtime_in_process():
    """Loading the library through the binding leaves exactly one HIP runtime
    mapped (the one PyTorch uses)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1806_04593_amd import yyg; yyg.lib()\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len(set(l.split()[-1] for l in maps if 'libamdhip64' in l)))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True)
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_status_strings():
    lib = yyg.lib()
    for s in (0, -1, -2, -3, -4, -5, -6, 7):
        assert isinstance(lib.yyg_status_string(s), bytes)


def _desc(res, lmax, r_edges=None):
    d = W.make_desc("t", np.linspace(0.0, 1.0, 9) if r_edges is None else r_edges, res, lmax, 1.0, 0)
    return d


def test_invalid_descriptors_rejected():
    bad = [
        dict(n_theta=0), dict(n_phi=-1), dict(lmax=-1), dict(lmax=yyg_cap() + 1),
        dict(delta_theta=-0.1), dict(delta_phi=math.pi / 4), dict(r_edges=np.array([0.0, 1.0, 1.0])),
        dict(r_edges=np.array([-1.0, 1.0])), dict(G=float("nan")),
    ]
    for change in bad:
        d = dict(_desc(5.0, 4))
        d.update(change)
        with pytest.raises(yyg.YygError) as ei:
            yyg.host_table(d, yyg.TABLE_WEIGHTS)
        assert ei.value.status == -1, change
        # plan creation validates before touching any device
        gd = yyg.make_desc(d["r_edges"], d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"], d["lmax"], d["G"])
        h = ctypes.c_void_p()
        assert yyg.lib().yyg_grid_create(ctypes.byref(gd), 0, ctypes.byref(h)) == -1
        assert not h.value


def test_wrong_table_size_and_null_handles():
    d = _desc(5.0, 4)
    gd = yyg.make_desc(d["r_edges"], d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"], d["lmax"], 1.0)
    out = np.zeros(10)
    assert yyg.lib().yyg_host_table(ctypes.byref(gd), yyg.TABLE_WEIGHTS, yyg._dptr(out), 10) == -1
    assert yyg.lib().yyg_host_table(ctypes.byref(gd), 99, yyg._dptr(out), 10) == -1
    lib = yyg.lib()
    assert lib.yyg_solve(None, None, 1, 0, None) == -1
    assert lib.yyg_upload_rho(None, None, 1, None) == -1
    assert lib.yyg_grid_destroy(None) == -1
    assert lib.yyg_grid_dims(None, None, None, None, None) == -1


def yyg_cap():
    return 128


@pytest.mark.parametrize("res", [15.0, 5.0, 2.0, 1.0])
def test_weights_match_oracle(res):
    d = _desc(res, 2)
    w = yyg.host_table(d, yyg.TABLE_WEIGHTS)
    th, ph = O.patch_edges(d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"])
    wo = O.overlap_weights(th, ph, d["delta_theta"], d["delta_phi"])
    # both sides sit within ~1e-13 of a 30-digit reference; small cells lose
    # a few digits to the cancellation between whole-cell and covered areas
    assert np.max(np.abs(w - wo)) < 1e-12
    assert abs(np.sum(O.solid_angles(th, ph) * w) - 2 * math.pi) < 1e-13


def test_weights_non_integer_span_and_zero_buffer():
    # 4 deg: 90/4 = 22.5 -> 25 cells with 5 deg buffers; and a grid without buffers
    for d in (_desc(4.0, 2), dict(_desc(5.0, 2), n_theta=18, n_phi=54, delta_theta=0.0, delta_phi=0.0)):
        w = yyg.host_table(d, yyg.TABLE_WEIGHTS)
        th, ph = O.patch_edges(d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"])
        wo = O.overlap_weights(th, ph, d["delta_theta"], d["delta_phi"])
        assert np.max(np.abs(w - wo)) < 1e-12


def _col_lm(L):
    cols = []
    for l in range(L + 1):
        cols.append((l, 0, 0))
        for m in range(1, l + 1):
            cols += [(l, m, 0), (l, m, 1)]
    return cols


@pytest.mark.parametrize("res,lmax", [(5.0, 24), (1.0, 64)])
def test_theta_table_matches_oracle(res, lmax):
    d = _desc(res, lmax)
    T = yyg.host_table(d, yyg.TABLE_THETA)
    th, _ = O.patch_edges(d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"])
    To = O.theta_integrals(th, lmax)
    for q, (l, m, s) in enumerate(_col_lm(lmax)):
        ref = To[:, l, m]
        assert np.max(np.abs(T[:, q] - ref)) <= 1e-12 * np.max(np.abs(ref)), (l, m)


def test_phi_table_matches_oracle():
    d = _desc(2.0, 25)
    CSt = yyg.host_table(d, yyg.TABLE_PHI)
    _, ph = O.patch_edges(d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"])
    C, S = O.phi_integrals(ph, 25)
    for q, (l, m, s) in enumerate(_col_lm(25)):
        ref = S[:, m] if s else C[:, m]
        assert np.max(np.abs(CSt[:, q] - ref)) < 1e-15


def test_cross_points_match_oracle():
    d = _desc(2.0, 1)
    X = yyg.host_table(d, yyg.TABLE_CROSS)
    th, ph = O.patch_edges(d["n_theta"], d["n_phi"], d["delta_theta"], d["delta_phi"])
    T, P = np.meshgrid(0.5 * (th[:-1] + th[1:]), 0.5 * (ph[:-1] + ph[1:]), indexing="ij")
    c, s, p = O.other_patch_angles(T.ravel(), P.ravel())
    np.testing.assert_allclose(X[:, 0], c, atol=1e-15)
    np.testing.assert_allclose(X[:, 1], s, atol=1e-15)
    np.testing.assert_allclose(X[:, 2], p, atol=1e-14)


@pytest.mark.parametrize("r_edges", [np.linspace(0.0, 1.0, 33), np.geomspace(1e5, 1e9, 61)])
def test_radial_recurrence_reproduces_direct_sums(r_edges):
    """Running the library's recurrence coefficients over random moments gives
    the oracle's direct double sums of Eqs. (19)-(20)."""
    L = 12
    d = _desc(5.0, L, r_edges)
    cf = yyg.host_table(d, yyg.TABLE_RADIAL)
    nR = len(r_edges) - 1
    rng = np.random.default_rng(3)
    AC = rng.normal(size=(2, nR, L + 1, L + 1))
    AS = rng.normal(size=(2, nR, L + 1, L + 1))
    UC, US = O.radial_sums(AC, AS, r_edges)
    for l in range(L + 1):
        a = AC[:, :, l, :]
        I = np.zeros_like(a[:, 0])
        Iv = np.zeros_like(a)
        for n in range(nR):
            I = cf[n, l, 0] * I + cf[n, l, 1] * a[:, n]
            Iv[:, n] = I
        Ov = np.zeros_like(a)
        Oc = np.zeros_like(a[:, 0])
        for n in range(nR - 1, -1, -1):
            an = a[:, n + 1] if n + 1 < nR else 0.0
            Oc = cf[n, l, 2] * Oc + cf[n, l, 3] * an
            Ov[:, n] = Oc
        U = Iv + Ov
        ref = UC[:, :, l, :]
        scale = np.max(np.abs(ref[:, :, : l + 1]), axis=1, keepdims=True) + 1e-300
        assert np.max(np.abs(U[:, :, : l + 1] - ref[:, :, : l + 1]) / scale) < 1e-12, l


@pytest.mark.parametrize("lmax", [4, 25, 64])
def test_rotation_blocks_rotate_the_harmonics(lmax):
    """D_l maps the normalised real harmonics (built here from the oracle's
    P_l^m and N^(lm)) at a point x to their values at R x, R the Yin <-> Yang
    map of Eqs. (23)-(24); each block is orthogonal."""
    d = _desc(5.0, lmax)
    D = yyg.host_table(d, yyg.TABLE_ROTATION)
    N = O.norm_factor(lmax)
    rng = np.random.default_rng(6)
    t = rng.uniform(0.1, 3.0, 30)
    p = rng.uniform(-3.1, 3.1, 30)

    def ybar(ct, st, ph):
        P = O.assoc_legendre(lmax, ct, st)
        out = []
        for l in range(lmax + 1):
            out.append(np.sqrt(N[l, 0]) * P[l, 0])
            for m in range(1, l + 1):
                out.append(np.sqrt(N[l, m]) * P[l, m] * np.cos(m * ph))
                out.append(np.sqrt(N[l, m]) * P[l, m] * np.sin(m * ph))
        return np.array(out)            # [Q, pts]
    Y = ybar(np.cos(t), np.sin(t), p)
    c2, s2, p2 = O.other_patch_angles(t, p)
    YR = ybar(c2, s2, p2)
    off = 0
    for l in range(lmax + 1):
        dd = 2 * l + 1
        blk = D[off:off + dd * dd].reshape(dd, dd)
        off += dd * dd
        q0 = l * l
        np.testing.assert_allclose(blk @ Y[q0:q0 + dd], YR[q0:q0 + dd], atol=1e-12)
        np.testing.assert_allclose(blk @ blk.T, np.eye(dd), atol=1e-12)


# ---------------------------------------------------------------------------
# full-sphere polar grid
# ---------------------------------------------------------------------------

def test_polar_tables_match_oracle():
    d = W.make_polar_desc("t", np.linspace(0.0, 1.0, 9), 5.0, 24, 1.0, 0)
    assert (d["n_theta"], d["n_phi"]) == (36, 72)
    w = yyg.host_table(d, yyg.TABLE_WEIGHTS)
    assert np.all(w == 1.0)
    th, ph = O.polar_edges(d["n_theta"], d["n_phi"])
    T = yyg.host_table(d, yyg.TABLE_THETA)
    To = O.theta_integrals(th, 24)
    CSt = yyg.host_table(d, yyg.TABLE_PHI)
    C, S = O.phi_integrals(ph, 24)
    for q, (l, m, s) in enumerate(_col_lm(24)):
        ref = To[:, l, m]
        assert np.max(np.abs(T[:, q] - ref)) <= 1e-12 * np.max(np.abs(ref)), (l, m)
        ref = S[:, m] if s else C[:, m]
        assert np.max(np.abs(CSt[:, q] - ref)) < 1e-14, (l, m, s)


def test_polar_descriptor_rules():
    d = W.make_polar_desc("t", np.linspace(0.0, 1.0, 9), 10.0, 4, 1.0, 0)
    with pytest.raises(yyg.YygError) as ei:
        yyg.host_table(d, yyg.TABLE_CROSS)          # there is no other patch
    assert ei.value.status == -5
    for change in (dict(delta_theta=0.01), dict(delta_phi=0.02), dict(kind=7)):
        bad = dict(d)
        bad.update(change)
        with pytest.raises(yyg.YygError) as ei:
            yyg.host_table(bad, yyg.TABLE_WEIGHTS)
        assert ei.value.status == -1, change


@pytest.mark.parametrize("kind,res", [("yinyang", 0.5), ("yinyang", 2.0), ("yinyang", 7.0), ("yinyang", 9.0),
                                      ("polar", 5.0), ("polar", 7.5)])
def test_mirror_symmetry_and_folded_phi_transform(kind, res):
    """The separable form folds each phi transform about the patch's central
    meridian (k -> n_phi - 1 - k): that needs the overlap weights even and
    the cos / sin cell integrals even / odd under the mirror, and then the
    contraction over n_phi cells equals the even / odd halves over
    ceil(n_phi / 2) (the middle cell, for odd n_phi, counted once)."""
    L = 12
    d = _desc(res, L) if kind == "yinyang" else W.make_polar_desc("p", np.linspace(0.0, 1.0, 3), res, L, 1.0, 0)
    nt, npp = d["n_theta"], d["n_phi"]
    w = yyg.host_table(d, yyg.TABLE_WEIGHTS).reshape(nt, npp)
    CS = yyg.host_table(d, yyg.TABLE_PHI).reshape(npp, -1)
    # a weight is a covered fraction: O(1) terms over the cell's solid
    # angle, whose rounding grows as the cells shrink (about 1.5e-12 at
    # 0.5 deg); the library folds up to 1e-10 and averages each mirror pair
    assert np.max(np.abs(w - w[:, ::-1])) <= (1e-12 if res >= 2.0 else 1e-10)
    cols = _col_lm(L)
    for q, (l, m, s) in enumerate(cols):
        sg = -1.0 if s else 1.0
        assert np.max(np.abs(CS[:, q] - sg * CS[::-1, q])) <= 1e-12 * max(1e-300, np.max(np.abs(CS[:, q])))
    # folded analysis of random rows against the plain contraction
    rng = np.random.default_rng(5)
    rho = rng.uniform(-1.0, 1.0, (7, nt, npp))
    h = (npp + 1) // 2
    half = np.ones(h)
    if npp % 2:
        half[-1] = 0.5
    wb = 0.5 * (w + w[:, ::-1])[:, :h] * half
    E = rho[..., :h] + rho[..., ::-1][..., :h]
    Od = rho[..., :h] - rho[..., ::-1][..., :h]
    for q, (l, m, s) in enumerate(cols):
        plain = np.einsum("rjk,jk,k->rj", rho, w, CS[:, q])
        folded = np.einsum("rjk,jk,k->rj", Od if s else E, wb, CS[:h, q])
        assert np.max(np.abs(folded - plain)) <= 1e-13 * np.max(np.abs(rho)) * npp, (l, m, s)
    # folded synthesis: even part plus / minus odd part at k and its mirror
    coef = rng.normal(size=(7, nt, len(cols)))
    plain = np.einsum("rjq,kq->rjk", coef, CS)
    ev = sum(np.einsum("rj,k->rjk", coef[..., q], CS[:h, q]) for q, c in enumerate(cols) if not c[2])
    od = sum(np.einsum("rj,k->rjk", coef[..., q], CS[:h, q]) for q, c in enumerate(cols) if c[2])
    back = np.concatenate([ev + od, (ev - od)[..., ::-1][..., npp % 2:]], axis=-1)
    # the mirror half uses CS[k] for CS[n_phi - 1 - k]: off by their asymmetry
    asym = sum(np.max(np.abs(coef[..., q])) * np.max(np.abs(CS[:, q] - (-1.0 if c[2] else 1.0) * CS[::-1, q]))
               for q, c in enumerate(cols))
    assert np.max(np.abs(back - plain)) <= 1e-13 * np.max(np.abs(plain)) + asym
