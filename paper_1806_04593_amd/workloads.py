"""Seeded synthetic density fields on the Yin-Yang grid.

This module places cells in space and evaluates analytic density recipes at
them.  It holds none of the solver's arithmetic (no weights, no Legendre
functions of the method, no moments, no radial sums); the C library and the
CPU oracle both take its output as their input.

Workloads (all FP64, numpy PCG64 seeded):

  small      n_R = 32 uniform shells on [0, 1], 5 deg patches (20 x 56),
             lmax 8, G = 1; volume fraction (4^3 sub-samples per cell) of the
             ball |x - (0.1, 0.05, 0)| <= 0.6 plus 0.01 U[0,1) noise per cell.
  sn_core    n_R = 400 log shells on [1e5, 1e9] cm, 2 deg (47 x 137), lmax 25;
             rho0(r) = 1e14 (1 + (r/1e6)^2)^-1.5 g/cm^3 times
             (1 + sum_{1<=l<=10} a_lm Y_lm), a_lm ~ N(0, 0.05^2).
  spheroid   n_R = 550 log shells on [1e5, 1e9] cm, 1 deg (92 x 272), lmax 40;
             rho0(r_s) with r_s^2 = x'^2 + y'^2 + (z'/0.7)^2 in a frame tilted
             20 deg about a seeded horizontal axis, times
             (1 + sum_{1<=l<=20} a_lm Y_lm), a_lm ~ N(0, 0.02^2).
  batch64    64 fields, n_R ~ U{100..600} uniform on [0, 1], resolution from
             {2, 3, 4} deg, lmax ~ U{10..30}, each built like `small`.
  binary     n_R = 1000 log shells on [1e5, 1e10] cm, 0.5 deg (182 x 542),
             lmax 64; rho0(r) + A g(x - x1) + 0.3 A g(x - x2), Gaussian cores
             of width 2e6 cm, A = 1e13 g/cm^3, separated by 2e7 cm along a
             seeded direction with the pair's centre of mass at the origin.

  polar_small, polar_sn_core
             the `small` and `sn_core` recipes on the full-sphere spherical
             polar grid (theta in [0, pi], phi in [0, 2 pi], one patch) at the
             same angular resolution: 36 x 72 and 90 x 180 cells.

The Yin patch frame is the global frame; a Yang cell with local angles
(theta, phi) sits at the global Cartesian point (-x', z', y') where
(x', y', z') are its local Cartesian coordinates.  The polar grid's frame is
the global frame.
"""

import math

import numpy as np
from scipy import special

G_CGS = 6.67430e-8

WORKLOADS = ("small", "sn_core", "spheroid", "binary", "polar_small", "polar_sn_core")


def grid_from_resolution(res_deg):
    """n = ceil(span/res) + 2 cells of `res` degrees per patch direction, the
    surplus split evenly into the two buffer widths.  Returns (n_theta,
    n_phi, delta_theta, delta_phi) with the widths in radians."""
    out = []
    for span in (90.0, 270.0):
        n = int(math.ceil(span / res_deg - 1e-9)) + 2
        out.append((n, math.radians((n * res_deg - span) / 2.0)))
    return out[0][0], out[1][0], out[0][1], out[1][1]


def make_desc(name, r_edges, res_deg, lmax, G, seed, recipe=None):
    n_t, n_p, d_t, d_p = grid_from_resolution(res_deg)
    return dict(name=name, kind="yinyang", patches=2, r_edges=np.asarray(r_edges, dtype=np.float64),
                n_theta=n_t, n_phi=n_p, delta_theta=d_t, delta_phi=d_p,
                lmax=int(lmax), G=float(G), res_deg=float(res_deg), seed=int(seed),
                recipe=recipe or name)


def make_polar_desc(name, r_edges, res_deg, lmax, G, seed, recipe=None):
    """Full-sphere polar grid: round(180/res) x round(360/res) cells."""
    n_t = int(round(180.0 / res_deg))
    n_p = int(round(360.0 / res_deg))
    return dict(name=name, kind="polar", patches=1, r_edges=np.asarray(r_edges, dtype=np.float64),
                n_theta=n_t, n_phi=n_p, delta_theta=0.0, delta_phi=0.0,
                lmax=int(lmax), G=float(G), res_deg=float(res_deg), seed=int(seed),
                recipe=recipe or name)


def describe(name):
    """Grid description of a named single-field workload."""
    if name == "small":
        return make_desc(name, np.linspace(0.0, 1.0, 33), 5.0, 8, 1.0, 1)
    if name == "sn_core":
        return make_desc(name, np.geomspace(1e5, 1e9, 401), 2.0, 25, G_CGS, 2)
    if name == "spheroid":
        return make_desc(name, np.geomspace(1e5, 1e9, 551), 1.0, 40, G_CGS, 3)
    if name == "binary":
        return make_desc(name, np.geomspace(1e5, 1e10, 1001), 0.5, 64, G_CGS, 5)
    if name == "polar_small":
        return make_polar_desc(name, np.linspace(0.0, 1.0, 33), 5.0, 8, 1.0, 1, recipe="small")
    if name == "polar_sn_core":
        return make_polar_desc(name, np.geomspace(1e5, 1e9, 401), 2.0, 25, G_CGS, 2, recipe="sn_core")
    raise ValueError(f"unknown workload {name!r}")


def batch_descs(n_fields=64, seed=4):
    """Uneven batch: sizes drawn with `seed`, field f seeded 1000 + f."""
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n_fields):
        n_r = int(rng.integers(100, 601))
        res = float(rng.choice([2.0, 3.0, 4.0]))
        lmax = int(rng.integers(10, 31))
        out.append(make_desc(f"batch{f}", np.linspace(0.0, 1.0, n_r + 1), res, lmax, 1.0, 1000 + f))
    return out


# ---------------------------------------------------------------------------
# cell placement
# ---------------------------------------------------------------------------

def _patch_edges(desc):
    n_t, n_p = desc["n_theta"], desc["n_phi"]
    if desc.get("kind", "yinyang") == "polar":
        return math.pi * np.arange(n_t + 1) / n_t, 2 * math.pi * np.arange(n_p + 1) / n_p
    d_t, d_p = desc["delta_theta"], desc["delta_phi"]
    th = (math.pi / 4 - d_t) + (math.pi / 2 + 2 * d_t) * np.arange(n_t + 1) / n_t
    ph = (-3 * math.pi / 4 - d_p) + (3 * math.pi / 2 + 2 * d_p) * np.arange(n_p + 1) / n_p
    return th, ph


def _to_global(patch, theta, phi):
    """Unit vectors (global frame) of local patch angles; shape (..., 3)."""
    x = np.sin(theta) * np.cos(phi)
    y = np.sin(theta) * np.sin(phi)
    z = np.cos(theta)
    if patch == 0:
        return np.stack([x, y, z], axis=-1)
    return np.stack([-x, z, y], axis=-1)


def n_patches(desc):
    return 1 if desc.get("kind", "yinyang") == "polar" else 2


def cell_directions(desc):
    """Global unit vector of every angular cell midpoint: [patches, n_theta, n_phi, 3]."""
    th, ph = _patch_edges(desc)
    tc, pc = 0.5 * (th[:-1] + th[1:]), 0.5 * (ph[:-1] + ph[1:])
    T, P = np.meshgrid(tc, pc, indexing="ij")
    return np.stack([_to_global(p, T, P) for p in range(n_patches(desc))])


def _real_sh(lmin, lmax, coeffs, dirs):
    """sum_{l,m} a_lm Y_lm(dir) with real orthonormal harmonics from SciPy."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    out = np.zeros(theta.shape)
    it = iter(coeffs)
    for l in range(lmin, lmax + 1):
        for m in range(-l, l + 1):
            Y = special.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                val = Y.real
            elif m > 0:
                val = math.sqrt(2.0) * (-1) ** m * Y.real
            else:
                val = math.sqrt(2.0) * (-1) ** m * Y.imag
            out += next(it) * val
    return out


def _n_coeffs(lmin, lmax):
    return sum(2 * l + 1 for l in range(lmin, lmax + 1))


def rho0(r):
    """Supernova-core envelope 1e14 (1 + (r/1e6)^2)^-1.5 g/cm^3."""
    return 1e14 * (1.0 + (r / 1e6) ** 2) ** -1.5


def _rotation(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def _ball_fraction(desc, rng, centre=(0.1, 0.05, 0.0), radius=0.6, sub=4):
    """Volume fraction of a ball in each cell from sub x sub x sub sub-cells
    (sub-cell midpoints weighted by their volumes)."""
    r = desc["r_edges"]
    th, ph = _patch_edges(desc)
    nR, n_t, n_p = len(r) - 1, desc["n_theta"], desc["n_phi"]
    u = (np.arange(sub) + 0.5) / sub
    ue = np.arange(sub + 1) / sub
    # sub-cell edges / midpoints
    ra, rb = r[:-1], r[1:]
    r_e = ra[:, None] + (rb - ra)[:, None] * ue[None, :]            # [nR, sub+1]
    r_m = 0.5 * (r_e[:, :-1] + r_e[:, 1:])
    vol_r = (r_e[:, 1:] ** 3 - r_e[:, :-1] ** 3) / 3.0               # [nR, sub]
    t_e = th[:-1, None] + (th[1:] - th[:-1])[:, None] * ue[None, :]
    t_m = 0.5 * (t_e[:, :-1] + t_e[:, 1:])
    vol_t = np.cos(t_e[:, :-1]) - np.cos(t_e[:, 1:])                 # [n_t, sub]
    p_m = ph[:-1, None] + (ph[1:] - ph[:-1])[:, None] * u[None, :]   # [n_p, sub]
    centre = np.asarray(centre)
    out = np.zeros((n_patches(desc), nR, n_t, n_p))
    for patch in range(n_patches(desc)):
        # global directions of sub-cell angular midpoints [n_t, st, n_p, sp, 3]
        T = t_m[:, :, None, None]
        P = p_m[None, None, :, :]
        d = _to_global(patch, np.broadcast_to(T, (n_t, sub, n_p, sub)),
                       np.broadcast_to(P, (n_t, sub, n_p, sub)))
        dc = d @ centre                                              # [n_t, st, n_p, sp]
        w_ang = np.broadcast_to(vol_t[:, :, None, None], dc.shape)
        for i in range(nR):
            acc = np.zeros((n_t, n_p))
            for s in range(sub):
                rr = r_m[i, s]
                dist2 = rr * rr - 2 * rr * dc + centre @ centre
                inside = (dist2 <= radius * radius).astype(np.float64)
                acc += vol_r[i, s] * (inside * w_ang).sum(axis=(1, 3))
            # every phi sub-cell has the same width, so the phi sum is a count
            tot = vol_r[i].sum() * vol_t.sum(axis=1)[:, None] * sub
            out[patch, i] = acc / tot
    out += 0.01 * rng.random(out.shape)
    return out


def density(desc):
    """Seeded FP64 density rho[patches, n_R, n_theta, n_phi] for a
    description made by `describe`, `batch_descs` or the desc builders."""
    name = desc.get("recipe", desc["name"])
    rng = np.random.default_rng(desc["seed"])
    r = desc["r_edges"]
    rc = 0.5 * (r[:-1] + r[1:])
    if name == "small" or name.startswith("batch"):
        return _ball_fraction(desc, rng)
    dirs = cell_directions(desc)                                     # [2, nt, np, 3]
    if name == "sn_core":
        a = rng.normal(0.0, 0.05, _n_coeffs(1, 10))
        pert = 1.0 + _real_sh(1, 10, a, dirs)                        # [2, nt, np]
        return rho0(rc)[None, :, None, None] * pert[:, None, :, :]
    if name == "spheroid":
        ang = rng.uniform(0.0, 2 * math.pi)
        R = _rotation((math.cos(ang), math.sin(ang), 0.0), math.radians(20.0))
        a = rng.normal(0.0, 0.02, _n_coeffs(1, 20))
        pert = 1.0 + _real_sh(1, 20, a, dirs)
        dl = dirs @ R.T                                              # tilted frame
        stretch = np.sqrt(dl[..., 0] ** 2 + dl[..., 1] ** 2 + (dl[..., 2] / 0.7) ** 2)
        out = np.empty((len(dirs), len(rc)) + pert.shape[1:])
        for p in range(len(dirs)):
            out[p] = rho0(rc[:, None, None] * stretch[p][None]) * pert[p][None]
        return out
    if name == "binary":
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        sep, q, A, sig = 2e7, 0.3, 1e13, 2e6
        x1 = v * sep * q / (1.0 + q)
        x2 = -v * sep / (1.0 + q)
        out = np.empty((len(dirs), len(rc)) + dirs.shape[1:3])
        for p in range(len(dirs)):
            d1 = dirs[p] @ x1
            d2 = dirs[p] @ x2
            for i, rr in enumerate(rc):
                g1 = np.exp(-(rr * rr - 2 * rr * d1 + x1 @ x1) / (2 * sig * sig))
                g2 = np.exp(-(rr * rr - 2 * rr * d2 + x2 @ x2) / (2 * sig * sig))
                out[p, i] = rho0(rr) + A * g1 + q * A * g2
        return out
    raise ValueError(f"unknown workload {name!r}")
