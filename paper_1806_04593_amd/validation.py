"""Homogeneous-ellipsoid validation of the solver (Sect. 5).

An ellipsoid of constant density with semi-axes a, b = 1.5 a, c = 2 a,
turned by pi/8 about the z axis so that the Yin and Yang patches see it
differently, fills a grid with equidistant shells out to r_max = c.  The
solver's potential at every output point (outer interface of every radial
cell, midpoint of every angular cell, both patches) is compared with the
semi-analytic potential of the ellipsoid (Chandrasekhar's formula with the
four integrals of Sect. 5 written as Carlson symmetric integrals); the
figure of merit is the maximum relative error over the whole domain.  The
paper sweeps lmax at a low (n_R 400, 2 degrees) and a high (n_R 800,
1 degree) resolution on the Yin-Yang and on the spherical polar grid.

This module builds the inputs (cell-averaged density: the volume fraction of
each cell inside the ellipsoid) and the reference potential, and runs the
sweep through the C library:

    python -m paper_1806_04593_amd.validation --res lr --lmax 0 10 20 40 80

It holds none of the solver's arithmetic.
"""

import argparse
import json
import math
import sys
import time

import numpy as np
from scipy import special

from . import workloads as W

DPHI = math.pi / 8


def axes(c=1.0):
    """Semi-axes (a, b, c) with b = 1.5 a and c = 2 a."""
    a = c / 2.0
    return a, 1.5 * a, c


def to_ellipsoid_frame(xyz):
    """Global (Yin-frame) Cartesian points -> ellipsoid frame: the paper
    adds pi/8 to the Yin longitude, i.e. turns the points by +pi/8 about z."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    cp, sp = math.cos(DPHI), math.sin(DPHI)
    return np.stack([cp * x - sp * y, sp * x + cp * y, z], axis=-1)


def ellipsoid_potential(xe, ye, ze, a, b, c, G=1.0, rho0=1.0):
    """Potential of the homogeneous ellipsoid at ellipsoid-frame points
    (vectorised).  pi G rho0 a b c (A x^2 + B y^2 + C z^2 - D) with
    A..D the integrals from u0 to infinity of Sect. 5, where u0 = 0 inside
    and the positive root of x^2/(a^2+u) + y^2/(b^2+u) + z^2/(c^2+u) = 1
    outside.  The integrals are Carlson's R_D and R_F:
    A = 2/3 R_D(b'^2, c'^2, a'^2), B = 2/3 R_D(a'^2, c'^2, b'^2),
    C = 2/3 R_D(a'^2, b'^2, c'^2), D = 2 R_F(a'^2, b'^2, c'^2), with
    a'^2 = a^2 + u0 etc."""
    xe, ye, ze = (np.asarray(v, dtype=np.float64) for v in (xe, ye, ze))
    x2, y2, z2 = xe * xe, ye * ye, ze * ze
    s2 = x2 / (a * a) + y2 / (b * b) + z2 / (c * c)
    u = np.zeros(s2.shape)
    out = s2 > 1.0
    if np.any(out):
        # f(u) = sum x^2/(a^2+u) - 1 is decreasing and convex: Newton from
        # u = 0 (f > 0) climbs monotonically to the root
        X, Y, Z = x2[out], y2[out], z2[out]
        v = np.zeros(X.shape)
        for _ in range(200):
            fa, fb, fc = a * a + v, b * b + v, c * c + v
            f = X / fa + Y / fb + Z / fc - 1.0
            df = -(X / fa ** 2 + Y / fb ** 2 + Z / fc ** 2)
            step = -f / df
            v = v + step
            # converged once the step is rounding noise on the scale of a^2 + u
            if np.all(np.abs(step) <= 4e-16 * (a * a + v)):
                break
        u[out] = v
    A2, B2, C2 = a * a + u, b * b + u, c * c + u
    Ai = 2.0 / 3.0 * special.elliprd(B2, C2, A2)
    Bi = 2.0 / 3.0 * special.elliprd(A2, C2, B2)
    Ci = 2.0 / 3.0 * special.elliprd(A2, B2, C2)
    Di = 2.0 * special.elliprf(A2, B2, C2)
    return math.pi * G * rho0 * a * b * c * (Ai * x2 + Bi * y2 + Ci * z2 - Di)


def _grid_desc(kind, n_r, res_deg, lmax, c=1.0):
    r = np.linspace(0.0, c, n_r + 1)
    if kind == "polar":
        return W.make_polar_desc(f"ellipsoid_polar_{n_r}_{res_deg:g}", r, res_deg, lmax, 1.0, 0)
    return W.make_desc(f"ellipsoid_yy_{n_r}_{res_deg:g}", r, res_deg, lmax, 1.0, 0)


def _edges(desc):
    return W._patch_edges(desc)


def volume_fraction(desc, sub=8, c=1.0):
    """Cell average of the unit-density ellipsoid: the fraction of each
    cell's volume inside it, [P, n_R, n_theta, n_phi].  Cells whose
    ellipsoidal radius s = sqrt((x/a)^2 + (y/b)^2 + (z/c)^2) at the centre
    is farther from 1 than the cell's extent allows (|grad s| <= 1/a) are
    fully inside or outside.  For the others the radial integral is exact:
    along a direction d the ellipsoid reaches R(d) = 1/s(d), so the inside
    part of the cell's radial range holds (min(R, r+)^3 - r-^3)/3 of volume
    per steradian; the angular integral is a sub x sub midpoint sum with the
    exact sin(theta) weights of the sub-cells."""
    a, b, c = axes(c)
    r = desc["r_edges"]
    th, ph = _edges(desc)
    P = W.n_patches(desc)
    nR, n_t, n_p = len(r) - 1, desc["n_theta"], desc["n_phi"]
    out = np.zeros((P, nR, n_t, n_p))
    rc = 0.5 * (r[:-1] + r[1:])
    tc, pc = 0.5 * (th[:-1] + th[1:]), 0.5 * (ph[:-1] + ph[1:])
    T, Pp = np.meshgrid(tc, pc, indexing="ij")
    dr = r[1:] - r[:-1]
    dth, dph = th[1] - th[0], ph[1] - ph[0]
    u = (np.arange(sub) + 0.5) / sub
    ue = np.arange(sub + 1) / sub
    for p in range(P):
        dirs = to_ellipsoid_frame(W._to_global(p, T, Pp))            # [n_t, n_p, 3]
        q = (dirs[..., 0] / a) ** 2 + (dirs[..., 1] / b) ** 2 + (dirs[..., 2] / c) ** 2
        for i in range(nR):
            s = rc[i] * np.sqrt(q)
            ext = (dr[i] + r[i + 1] * (dth + dph)) / a               # bound on the variation of s
            inside = s + 0.5 * ext < 1.0
            cut = np.abs(s - 1.0) <= 0.5 * ext
            out[p, i][inside] = 1.0
            js, ks = np.nonzero(cut)
            if js.size == 0:
                continue
            te = th[js][:, None] + dth * ue[None, :]
            tm = 0.5 * (te[:, :-1] + te[:, 1:])
            vt = np.cos(te[:, :-1]) - np.cos(te[:, 1:])               # [n, sub]
            pm = ph[ks][:, None] + dph * u[None, :]                    # [n, sub]
            n = js.size
            Tm = np.broadcast_to(tm[:, :, None], (n, sub, sub))
            Pm = np.broadcast_to(pm[:, None, :], (n, sub, sub))
            d = to_ellipsoid_frame(W._to_global(p, Tm, Pm))            # [n, sub, sub, 3]
            R = 1.0 / np.sqrt((d[..., 0] / a) ** 2 + (d[..., 1] / b) ** 2 + (d[..., 2] / c) ** 2)
            lo, hi = r[i], r[i + 1]
            vin = (np.clip(R, lo, hi) ** 3 - lo ** 3) / 3.0            # inside volume per steradian
            acc = np.sum(vin * vt[:, :, None], axis=(1, 2)) / sub
            full = (hi ** 3 - lo ** 3) / 3.0 * vt.sum(axis=1)
            out[p, i, js, ks] = np.minimum(acc / full, 1.0)
    return out


def reference_potential(desc, c=1.0, G=1.0):
    """Semi-analytic potential at every output point: outer interface
    r_(n+1), angular cell midpoint, every patch; [P, n_R, n_theta, n_phi]."""
    a, b, cc = axes(c)
    r = desc["r_edges"]
    th, ph = _edges(desc)
    tc, pc = 0.5 * (th[:-1] + th[1:]), 0.5 * (ph[:-1] + ph[1:])
    T, Pp = np.meshgrid(tc, pc, indexing="ij")
    P = W.n_patches(desc)
    out = np.zeros((P, len(r) - 1, desc["n_theta"], desc["n_phi"]))
    for p in range(P):
        dirs = to_ellipsoid_frame(W._to_global(p, T, Pp))
        for n in range(len(r) - 1):
            x = r[n + 1] * dirs
            out[p, n] = ellipsoid_potential(x[..., 0], x[..., 1], x[..., 2], a, b, cc, G)
    return out


def ellipsoidal_radius(desc, c=1.0):
    """s = sqrt((x/a)^2 + (y/b)^2 + (z/c)^2) at every output point."""
    a, b, cc = axes(c)
    r = desc["r_edges"]
    th, ph = _edges(desc)
    tc, pc = 0.5 * (th[:-1] + th[1:]), 0.5 * (ph[:-1] + ph[1:])
    T, Pp = np.meshgrid(tc, pc, indexing="ij")
    P = W.n_patches(desc)
    out = np.zeros((P, len(r) - 1, desc["n_theta"], desc["n_phi"]))
    for p in range(P):
        d = to_ellipsoid_frame(W._to_global(p, T, Pp))
        q = np.sqrt((d[..., 0] / a) ** 2 + (d[..., 1] / b) ** 2 + (d[..., 2] / cc) ** 2)
        out[p] = r[1:, None, None] * q[None]
    return out


def sweep(kinds, setups, lmaxes, method="separable", log=print):
    """Run the solver over grids x lmax; returns a list of result rows."""
    import torch

    from . import yyg
    rows = []
    for kind in kinds:
        for name, (n_r, res) in setups.items():
            base = _grid_desc(kind, n_r, res, 0)
            t0 = time.perf_counter()
            rho = volume_fraction(base)
            ref = reference_potential(base)
            srad = ellipsoidal_radius(base)
            log(f"[validate] {kind} {name}: n_r={n_r} {base['n_theta']}x{base['n_phi']}, inputs in "
                f"{time.perf_counter() - t0:.1f} s")
            d_rho = torch.from_numpy(rho).to("cuda:0")
            d_phi = torch.empty(rho.shape, dtype=torch.float64, device="cuda:0")
            near = np.abs(srad - 1.0) < 0.05
            core = srad < 0.5
            for L in lmaxes:
                desc = _grid_desc(kind, n_r, res, L)
                g = yyg.Grid(desc, 0)
                g.set_method(method)
                g.upload_rho(d_rho)
                g.solve(d_phi)
                torch.cuda.synchronize()
                phi = d_phi.cpu().numpy()
                rel = np.abs(phi - ref) / np.abs(ref)
                row = {"grid": kind, "setup": name, "n_r": n_r, "res_deg": res, "lmax": L,
                       "max_rel_err": float(rel.max()),
                       "max_rel_err_near_surface": float(rel[near].max()) if near.any() else None,
                       "max_rel_err_core": float(rel[core].max()) if core.any() else None}
                rows.append(row)
                log(f"[validate] {kind} {name} lmax {L}: max rel err {row['max_rel_err']:.3e} "
                    f"(|s-1|<0.05: {row['max_rel_err_near_surface']:.3e}, s<0.5: {row['max_rel_err_core']:.3e})")
                g.close()
            del d_rho, d_phi
    return rows


SETUPS = {"lr": (400, 2.0), "hr": (800, 1.0)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--res", nargs="+", default=["lr", "hr"], choices=sorted(SETUPS))
    ap.add_argument("--grids", nargs="+", default=["yinyang", "polar"], choices=("yinyang", "polar"))
    ap.add_argument("--lmax", nargs="+", type=int, default=[0, 5, 10, 20, 40, 60, 80])
    ap.add_argument("--method", default="separable", choices=("dense", "separable"))
    ap.add_argument("--json", default=None, help="write the rows to this file")
    a = ap.parse_args(argv)
    rows = sweep(a.grids, {k: SETUPS[k] for k in a.res}, a.lmax, a.method,
                 log=lambda m: print(m, file=sys.stderr, flush=True))
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(rows, fh, indent=1)
    print(json.dumps(rows))


if __name__ == "__main__":
    main()
