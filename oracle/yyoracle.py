"""Plain FP64 CPU oracle of the Yin-Yang multipole gravity solver.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports, calls or links anything here.

Every function cites the passage of Almanstoetter et al. (2018) it follows.
Sect. 2 gives the multipole method on a spherical polar grid (Eqs. 1-18, the
appendix recurrences A1-A7), Sect. 3 its separation into angular moments
(Eqs. 19-22), Sect. 4 the Yin-Yang version (Eqs. 23-29).

Readings taken where the paper is silent, garbled or ambiguous (each is also
listed in the design notes of the repository):

* Eq. (A4) is printed with a misplaced bracket; the closed form used here is
  T^(22) = 1/4 [(cos 3t+ - cos 3t-) - 9 (cos t+ - cos t-)], the integral of
  3 sin^3 t (checked by the tests against quadrature).
* Eq. (24) gives phi_Yang through an arctan whose quadrant is not fixed; the
  only choice that makes the map its own inverse (as Sect. 4 states) is
  phi_Yang = atan2(cos t, -sin t cos p), i.e. the Cartesian map
  (x, y, z) -> (-x, z, y).
* The partial-cell surface weights w_jk (Sect. 4, Eq. 25) are the exact
  fraction of the cell's solid angle that the other patch does not cover,
  counted once, plus one half of the covered fraction: w = 1 - f/2.
* The angular evaluation point of a cell is its midpoint (theta_c, phi_c); the
  radial evaluation points are the outer interfaces r_n, n = 1..n_R (Sect. 2,
  after Eq. 13).
* Eqs. (16)-(17) overflow double precision at large l and r; they are
  evaluated here in the algebraically identical ratio forms
  R_in,i / r_n^(l+1) and r_n^l R_out,i, using expm1/log to avoid cancellation.

Range: the unnormalised P_l^m of Eq. (A3) and the factorial ratios of
Eq. (8) leave FP64's range together near lmax 90 (their product overflows
in the synthesis); the oracle is used up to lmax 80.

Array conventions: rho and phi are [2][n_R][n_theta][n_phi] (patch 0 = Yin,
patch 1 = Yang, each in its own local coordinates); moment and radial arrays
are indexed [patch, shell or interface, l, m].  The full-sphere spherical
polar grid of Sect. 2 (the method before the Yin-Yang extension) is the
single-patch case: rho and phi are [1][n_R][n_theta][n_phi] over
theta in [0, pi], phi in [0, 2 pi], every cell counted once (no weights).
"""

import math
import warnings

import numpy as np
from scipy import integrate

__all__ = [
    "patch_dims_from_resolution", "patch_edges", "solid_angles",
    "other_patch_angles", "overlap_weights", "assoc_legendre",
    "theta_integrals", "phi_integrals", "norm_factor", "moments",
    "radial_in_ratio", "radial_out_ratio", "radial_sums",
    "potential_at", "solve", "solve_sampled",
    "polar_edges", "potential_polar_at", "solve_polar", "solve_polar_sampled",
]


# ---------------------------------------------------------------------------
# Grid geometry (Sect. 4: the two congruent patches and their intervals)
# ---------------------------------------------------------------------------

def patch_dims_from_resolution(res_deg):
    """Cell counts and buffer widths of one patch for a target resolution.

    The paper fixes the patch intervals theta in [pi/4 - d_t, 3pi/4 + d_t],
    phi in [-3pi/4 - d_p, 3pi/4 + d_p] (Sect. 4) but not how n and the buffer
    widths follow from a resolution.  Convention used here: n = ceil(span /
    res) + 2 cells of exactly `res` degrees, the buffer being (n res - span)/2
    on each side.  Returns (n_theta, n_phi, delta_theta, delta_phi) in
    radians.
    """
    out = []
    for span in (90.0, 270.0):
        n = int(math.ceil(span / res_deg - 1e-9)) + 2
        out.append((n, math.radians((n * res_deg - span) / 2.0)))
    (n_t, d_t), (n_p, d_p) = out
    return n_t, n_p, d_t, d_p


def patch_edges(n_theta, n_phi, delta_theta, delta_phi):
    """Equidistant cell edges of one patch (Sect. 4, patch intervals)."""
    t0, t1 = math.pi / 4 - delta_theta, 3 * math.pi / 4 + delta_theta
    p0, p1 = -3 * math.pi / 4 - delta_phi, 3 * math.pi / 4 + delta_phi
    theta = t0 + (t1 - t0) * np.arange(n_theta + 1) / n_theta
    phi = p0 + (p1 - p0) * np.arange(n_phi + 1) / n_phi
    return theta, phi


def solid_angles(theta_edges, phi_edges):
    """Cell solid angles (cos t- - cos t+)(p+ - p-), the factor of Eq. (25)."""
    dcos = np.cos(theta_edges[:-1]) - np.cos(theta_edges[1:])
    dphi = phi_edges[1:] - phi_edges[:-1]
    return dcos[:, None] * dphi[None, :]


def other_patch_angles(theta, phi):
    """Angles of a point in the other patch's frame (Eqs. 23-24).

    Returns (cos t', sin t', p').  cos t' = sin t sin p is Eq. (23) itself;
    sin t' is the non-negative root sqrt(1 - cos^2 t'), evaluated as
    hypot(cos t, sin t cos p) which is the same number without the
    cancellation near the other patch's poles; p' follows Eq. (24) with the
    quadrant that makes the map an involution (see module docstring).
    """
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    cos_t2 = st * sp
    sin_t2 = np.hypot(ct, st * cp)
    phi2 = np.arctan2(ct, -st * cp)
    return cos_t2, sin_t2, phi2


def _exclusion_half_width(phi, c, t):
    """Half width e(p) of the theta band around pi/2 that the other patch
    leaves uncovered along the meridian p of this patch.

    A point lies in the other patch iff its other-frame colatitude is inside
    [pi/4 - d_t, 3pi/4 + d_t], i.e. |sin t sin p| <= c = cos(pi/4 - d_t), and
    its other-frame longitude is inside [-3pi/4 - d_p, 3pi/4 + d_p], which
    fails iff cos p > 0 and |cos t| < sin t cos p tan(pi/4 - d_p).  Both
    failure sets are theta bands centred on pi/2; e is the wider half width.
    """
    s = abs(math.sin(phi))
    e1 = 0.0
    if s > c:
        e1 = math.pi / 2 - math.asin(c / s)
    e2 = 0.0
    cp = math.cos(phi)
    if cp > 0.0 and t > 0.0:
        e2 = math.atan(t * cp)
    return max(e1, e2)


def overlap_weights(theta_edges, phi_edges, delta_theta, delta_phi):
    """Surface weights w_jk of Sect. 4 (Eq. 25).

    w = 1 where the other patch does not reach, 1/2 where it covers the cell,
    and for cut cells 1 - f/2 with f the covered fraction of the solid angle.
    The paper computes cut cells "numerically" without giving the method;
    here f is the exact area: along each meridian the covered theta-range is
    known in closed form (see _exclusion_half_width), so the inner integral
    of sin t is a difference of cosines and the phi integral is done by
    adaptive Gauss-Kronrod quadrature (QUADPACK) with the kinks as
    breakpoints.  Identical on both patches (Sect. 4).
    """
    c = math.cos(math.pi / 4 - delta_theta)
    t = math.tan(math.pi / 4 - delta_phi)
    n_t, n_p = len(theta_edges) - 1, len(phi_edges) - 1
    omega = solid_angles(theta_edges, phi_edges)
    f = np.zeros((n_t, n_p))

    def e_range(pa, pb):
        # e grows with |sin p| (first band) and with max(cos p, 0) (second),
        # so its extremes over [pa, pb] sit at the ends or at multiples of
        # pi/2 inside.
        cand = [pa, pb] + [k * math.pi / 2 for k in range(-4, 5)
                           if pa < k * math.pi / 2 < pb]
        s_vals = [abs(math.sin(x)) for x in cand]
        c_vals = [max(math.cos(x), 0.0) for x in cand]
        e1 = lambda s: math.pi / 2 - math.asin(c / s) if s > c else 0.0
        e2 = lambda cc: math.atan(t * cc) if (cc > 0 and t > 0) else 0.0
        e_max = max(e1(max(s_vals)), e2(max(c_vals)))
        e_low = max(e1(min(s_vals)), e2(min(c_vals)))  # lower bound of min e
        return e_low, e_max

    for k in range(n_p):
        pa, pb = phi_edges[k], phi_edges[k + 1]
        e_low, e_max = e_range(pa, pb)
        # breakpoints where the integrand is not smooth
        pts = set()
        for base in (math.asin(min(c, 1.0)), math.pi / 2):
            for x in (base, -base, math.pi - base, -math.pi + base):
                if pa < x < pb:
                    pts.add(x)
        for j in range(n_t):
            ta, tb = theta_edges[j], theta_edges[j + 1]
            d = 0.0 if ta <= math.pi / 2 <= tb else min(abs(ta - math.pi / 2), abs(tb - math.pi / 2))
            dd = max(abs(ta - math.pi / 2), abs(tb - math.pi / 2))
            full = math.cos(ta) - math.cos(tb)
            if e_max <= d:
                f[j, k] = 1.0
                continue
            if e_low >= dd:
                f[j, k] = 0.0
                continue

            def covered(ph):
                e = _exclusion_half_width(ph, c, t)
                lo, hi = max(ta, math.pi / 2 - e), min(tb, math.pi / 2 + e)
                excl = math.cos(lo) - math.cos(hi) if hi > lo else 0.0
                return full - excl

            cell_pts = set(pts)
            for v in (d, dd):  # where the band edge crosses theta- or theta+
                if v > 0:
                    cv = math.cos(v)
                    if cv > 0 and c / cv <= 1.0:
                        s = c / cv
                        for x in (math.asin(s), -math.asin(s), math.pi - math.asin(s), -math.pi + math.asin(s)):
                            if pa < x < pb:
                                cell_pts.add(x)
                    if t > 0:
                        cc = math.tan(v) / t
                        if cc <= 1.0:
                            for x in (math.acos(cc), -math.acos(cc)):
                                if pa < x < pb:
                                    cell_pts.add(x)
            with warnings.catch_warnings():
                # at a few coarse-grid cut cells QUADPACK's own error estimate
                # (~1e-12) stays above the 1e-14 asked and it warns; those
                # values sit within 8e-13 of a 20-digit reference of the
                # covered fraction (tests/test_weights_mpmath.py)
                warnings.simplefilter("ignore", integrate.IntegrationWarning)
                val, _ = integrate.quad(covered, pa, pb, points=sorted(cell_pts) or None,
                                        epsabs=1e-16, epsrel=1e-14, limit=400)
            f[j, k] = val / omega[j, k]
    return 1.0 - 0.5 * f


# ---------------------------------------------------------------------------
# Polar and azimuthal integrals (Sect. 2, Eqs. 13-18 and the appendix)
# ---------------------------------------------------------------------------

def assoc_legendre(lmax, x, s):
    """Unnormalised associated Legendre functions P_l^m(x), 0 <= m <= l <= lmax,
    with the Condon-Shortley phase implied by Eq. (A3).  `s` = sqrt(1 - x^2)
    >= 0 is passed in so callers can supply it without cancellation.
    Returns P[l, m, ...] (zero for m > l).  Standard three-term recurrence in
    l at fixed m, seeded by the sectoral values.
    """
    x = np.asarray(x, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    P = np.zeros((lmax + 1, lmax + 1) + x.shape)
    P[0, 0] = 1.0
    for m in range(1, lmax + 1):
        P[m, m] = -(2 * m - 1) * s * P[m - 1, m - 1]
    for m in range(0, lmax):
        P[m + 1, m] = (2 * m + 1) * x * P[m, m]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            P[l, m] = ((2 * l - 1) * x * P[l - 1, m] - (l + m - 1) * P[l - 2, m]) / (l - m)
    return P


def theta_integrals(theta_edges, lmax):
    """T_j^(lm) of Eq. (18), by the recurrences (A1)-(A7) in the appendix's
    order.  Returns T[j, l, m] for 0 <= m <= l <= lmax (zero for m > l).
    (A4) is taken in the corrected form stated in the module docstring.
    """
    ta, tb = theta_edges[:-1], theta_edges[1:]          # theta_j^-, theta_j^+
    xa, xb = np.cos(ta), np.cos(tb)
    sa, sb = np.sin(ta), np.sin(tb)
    Pa = assoc_legendre(lmax + 1, xa, sa)
    Pb = assoc_legendre(lmax + 1, xb, sb)
    n = len(ta)
    T = np.zeros((lmax + 1, lmax + 1, n))
    # (A1)
    T[0, 0] = Pa[1, 0] - Pb[1, 0]
    # (A2), l > 0
    for l in range(1, lmax + 1):
        T[l, 0] = (Pb[l - 1, 0] - Pa[l - 1, 0] + Pa[l + 1, 0] - Pb[l + 1, 0]) / (2 * l + 1)
    if lmax >= 1:
        # (A3)
        T[1, 1] = 0.5 * (ta - tb + 0.5 * (np.sin(2 * tb) - np.sin(2 * ta)))
    if lmax >= 2:
        # (A4), corrected bracket
        T[2, 2] = 0.25 * ((np.cos(3 * tb) - np.cos(3 * ta)) - 9.0 * (np.cos(tb) - np.cos(ta)))
    # (A5), l >= 3
    for l in range(3, lmax + 1):
        T[l, l] = (xa * Pa[l, l] - xb * Pb[l, l]
                   + l * (2 * l - 3) * (2 * l - 1) * T[l - 2, l - 2]) / (l + 1)
    # (A6), l >= 2 (l = 1 is covered by A2)
    for l in range(2, lmax + 1):
        T[l, l - 1] = -(sb * Pb[l, l] - sa * Pa[l, l]) / (l + 1)
    # (A7), 1 <= m <= l - 2
    for l in range(3, lmax + 1):
        for m in range(1, l - 1):
            T[l, m] = ((2 * l - 1) * (sb ** 2 * Pb[l - 1, m] - sa ** 2 * Pa[l - 1, m])
                       + (l - 2) * (l + m - 1) * T[l - 2, m]) / ((l + 1) * (l - m))
    return np.moveaxis(T, 2, 0)


def phi_integrals(phi_edges, lmax):
    """C_k^(m) and S_k^(m) of Eqs. (14)-(15).  Returns (C[k, m], S[k, m])."""
    pa, pb = phi_edges[:-1], phi_edges[1:]
    n = len(pa)
    C = np.zeros((n, lmax + 1))
    S = np.zeros((n, lmax + 1))
    C[:, 0] = pb - pa
    for m in range(1, lmax + 1):
        C[:, m] = (np.sin(m * pb) - np.sin(m * pa)) / m
        S[:, m] = (np.cos(m * pa) - np.cos(m * pb)) / m
    return C, S


def norm_factor(lmax):
    """N^(lm) = (l-m)!/(l+m)! * 2/delta^(m), Eqs. (8)-(9).  Returns N[l, m]."""
    N = np.zeros((lmax + 1, lmax + 1))
    for l in range(lmax + 1):
        for m in range(l + 1):
            # (l-m)!/(l+m)! as a product of exact reciprocals
            ratio = 1.0
            for v in range(l - m + 1, l + m + 1):
                ratio /= v
            N[l, m] = ratio * (1.0 if m == 0 else 2.0)
    return N


# ---------------------------------------------------------------------------
# Angular moments (Sect. 3 Eqs. 21-22, Sect. 4 Eqs. 26-27)
# ---------------------------------------------------------------------------

def moments(rho, w, T, C, S):
    """A_C and A_S of Eqs. (26)-(27) for both patches.

    rho[p, i, j, k], w[j, k], T[j, l, m], C[k, m], S[k, m] ->
    (A_C[p, i, l, m], A_S[p, i, l, m]).  The double sum runs over k inside
    j, as written; w, T, C and S are the same on both patches (Sect. 4).
    """
    rw = rho * w[None, None, :, :]
    XC = rw @ C                     # sum over k: [p, i, j, m]
    XS = rw @ S
    AC = np.einsum("pijm,jlm->pilm", XC, T, optimize=True)
    AS = np.einsum("pijm,jlm->pilm", XS, T, optimize=True)
    return AC, AS


# ---------------------------------------------------------------------------
# Radial sums (Sect. 2 Eqs. 11-12, 16-17; Sect. 3 Eqs. 19-20)
# ---------------------------------------------------------------------------

def radial_in_ratio(l, r_lo, r_hi, r_n):
    """R_in^(l) of Eq. (16) over [r_lo, r_hi], divided by r_n^(l+1)
    (r_hi <= r_n).  Identity used:
    (r_hi^(l+3) - r_lo^(l+3)) / ((l+3) r_n^(l+1))
      = r_n^2 (r_hi/r_n)^(l+3) (1 - (r_lo/r_hi)^(l+3)) / (l+3).
    """
    r_lo, r_hi, r_n = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (r_lo, r_hi, r_n)))
    q = np.where(r_lo > 0, r_lo / np.where(r_hi > 0, r_hi, 1.0), 0.0)
    with np.errstate(divide="ignore"):
        frac = np.where(q > 0, -np.expm1((l + 3) * np.log(np.where(q > 0, q, 1.0))), 1.0)
    return r_n ** 2 * (r_hi / r_n) ** (l + 3) * frac / (l + 3)


def radial_out_ratio(l, r_lo, r_hi, r_n):
    """R_out^(l) of Eq. (17) over [r_lo, r_hi], multiplied by r_n^l
    (0 < r_n <= r_lo).  Identity used, with q = r_lo/r_hi:
    l != 2: r_n^2 (r_n/r_lo)^(l-2) (1 - q^(l-2)) / (l-2);
    l == 2: r_n^2 ln(r_hi/r_lo).
    """
    r_lo, r_hi, r_n = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (r_lo, r_hi, r_n)))
    lq = np.log(r_lo / r_hi)
    if l == 2:
        return -r_n ** 2 * lq
    return r_n ** 2 * (r_n / r_lo) ** (l - 2) * (-np.expm1((l - 2) * lq)) / (l - 2)


def radial_sums(AC, AS, r_edges):
    """U = Phi_in + Phi_out coefficients of Eqs. (19)-(20) at every outer
    interface r_n, n = 1..n_R, before the factor cos/sin(m phi).

    U_X[p, n-1, l, m] = sum_{i<=n} R_in,i/r_n^(l+1) A_X[p,i] + sum_{i>n} r_n^l R_out,i A_X[p,i]
    as plain double sums over shells (no recurrence).
    """
    r = np.asarray(r_edges, dtype=np.float64)
    nR = len(r) - 1
    lmax = AC.shape[2] - 1
    UC = np.zeros_like(AC)
    US = np.zeros_like(AS)
    n_idx = np.arange(1, nR + 1)[:, None]     # interface n (row)
    i_idx = np.arange(1, nR + 1)[None, :]     # cell i (column)
    r_n = r[n_idx]
    r_lo, r_hi = r[i_idx - 1], r[i_idx]
    inner = i_idx <= n_idx
    for l in range(lmax + 1):
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            Win = np.where(inner, radial_in_ratio(l, r_lo, r_hi, r_n), 0.0)
            Wout = np.where(~inner, radial_out_ratio(l, np.where(inner, 1.0, r_lo),
                                                     np.where(inner, 2.0, r_hi), r_n), 0.0)
        W = Win + Wout                                   # [n, i]
        m = slice(0, l + 1)
        UC[:, :, l, m] = np.einsum("ni,pim->pnm", W, AC[:, :, l, m])
        US[:, :, l, m] = np.einsum("ni,pim->pnm", W, AS[:, :, l, m])
    return UC, US


# ---------------------------------------------------------------------------
# Synthesis and patch combination (Eq. 5, Eqs. 19-20, Eqs. 28-29)
# ---------------------------------------------------------------------------

def potential_at(UC, US, G, p, n, theta, phi, chunk=4096):
    """Phi at points given by target patch p, interface index n (0-based,
    i.e. r_(n+1)) and local angles (theta, phi) of patch p (Eqs. 28-29).

    Phi = -G sum_{l,m} N^(lm) [P_l^m(cos t)(cos m p U_C[p] + sin m p U_S[p])
                              + P_l^m(cos t')(cos m p' U_C[pbar] + sin m p' U_S[pbar])]
    with (t', p') the same point in the other patch's frame (Eqs. 23-24).
    All arguments are 1-D arrays of equal length (p, n integer).
    """
    p = np.asarray(p)
    n = np.asarray(n)
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    if theta.size > chunk:
        # points are independent: the same sums, a bounded chunk of points at
        # a time (the P table is (lmax+1)^2 values per point)
        out = np.empty(theta.shape)
        for i in range(0, theta.size, chunk):
            sl = slice(i, i + chunk)
            out[sl] = potential_at(UC, US, G, p[sl], n[sl], theta[sl], phi[sl], chunk)
        return out
    lmax = UC.shape[2] - 1
    N = norm_factor(lmax)
    m = np.arange(lmax + 1)
    out = np.zeros(theta.shape)
    frames = ((np.cos(theta), np.sin(theta), phi, p),
              other_patch_angles(theta, phi) + (1 - p,))
    for x, s, ph, src in frames:
        P = assoc_legendre(lmax, x, s)                  # [l, m, pts]
        cm = np.cos(m[:, None] * ph[None, :])           # [m, pts]
        sm = np.sin(m[:, None] * ph[None, :])
        uc = np.moveaxis(UC[src, n], 0, -1)             # [l, m, pts]
        us = np.moveaxis(US[src, n], 0, -1)
        out += np.einsum("lm,lmx->x", N, P * (cm[None] * uc + sm[None] * us))
    return -G * out


def _tables(r_edges, n_theta, n_phi, delta_theta, delta_phi, lmax):
    th, ph = patch_edges(n_theta, n_phi, delta_theta, delta_phi)
    w = overlap_weights(th, ph, delta_theta, delta_phi)
    T = theta_integrals(th, lmax)
    C, S = phi_integrals(ph, lmax)
    return th, ph, w, T, C, S


def solve(r_edges, n_theta, n_phi, delta_theta, delta_phi, lmax, G, rho, tables=None):
    """Full solve: rho[2, n_R, n_theta, n_phi] -> Phi[2, n_R, n_theta, n_phi]
    at the outer radial interfaces and the angular cell midpoints."""
    th, ph, w, T, C, S = tables or _tables(r_edges, n_theta, n_phi, delta_theta, delta_phi, lmax)
    AC, AS = moments(rho, w, T, C, S)
    UC, US = radial_sums(AC, AS, r_edges)
    nR = len(r_edges) - 1
    tc = 0.5 * (th[:-1] + th[1:])
    pc = 0.5 * (ph[:-1] + ph[1:])
    TT, PP = np.meshgrid(tc, pc, indexing="ij")
    tt, pp = TT.ravel(), PP.ravel()
    out = np.zeros((2, nR, n_theta * n_phi))
    for p in range(2):
        for n in range(nR):
            out[p, n] = potential_at(UC, US, G, np.full(tt.shape, p), np.full(tt.shape, n), tt, pp)
    return out.reshape(2, nR, n_theta, n_phi)


def solve_sampled(r_edges, n_theta, n_phi, delta_theta, delta_phi, lmax, G, rho,
                  samples, tables=None, return_moments=False):
    """Phi at selected outputs only.  samples: int array [S, 4] of
    (p, n, j, k) with n the 0-based interface index.  The moments and radial
    sums are computed in full (every output depends on all of rho); only the
    synthesis is restricted to the samples."""
    th, ph, w, T, C, S = tables or _tables(r_edges, n_theta, n_phi, delta_theta, delta_phi, lmax)
    AC, AS = moments(rho, w, T, C, S)
    UC, US = radial_sums(AC, AS, r_edges)
    samples = np.asarray(samples)
    tc = 0.5 * (th[:-1] + th[1:])
    pc = 0.5 * (ph[:-1] + ph[1:])
    vals = potential_at(UC, US, G, samples[:, 0], samples[:, 1], tc[samples[:, 2]], pc[samples[:, 3]])
    if return_moments:
        return vals, (AC, AS)
    return vals


# ---------------------------------------------------------------------------
# Full-sphere spherical polar grid (Sect. 2): the single-patch method
# ---------------------------------------------------------------------------

def polar_edges(n_theta, n_phi):
    """Equidistant cell edges of the spherical polar grid of Sect. 2:
    theta in [0, pi], phi in [0, 2 pi]."""
    theta = math.pi * np.arange(n_theta + 1) / n_theta
    phi = 2.0 * math.pi * np.arange(n_phi + 1) / n_phi
    return theta, phi


def _polar_tables(n_theta, n_phi, lmax):
    th, ph = polar_edges(n_theta, n_phi)
    w = np.ones((n_theta, n_phi))        # each cell covers its solid angle once
    T = theta_integrals(th, lmax)
    C, S = phi_integrals(ph, lmax)
    return th, ph, w, T, C, S


def potential_polar_at(UC, US, G, n, theta, phi):
    """Phi of Eq. (5) on the polar grid: the coefficients of Eqs. (19)-(20)
    (interface index n, 0-based) times N^(lm) P_l^m(cos t)(cos m p, sin m p),
    summed over l <= lmax, m <= l.  There is a single frame and no patch
    combination.  UC, US are [1, n_R, l, m]; n, theta, phi are 1-D arrays."""
    n = np.asarray(n)
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lmax = UC.shape[2] - 1
    N = norm_factor(lmax)
    m = np.arange(lmax + 1)
    P = assoc_legendre(lmax, np.cos(theta), np.sin(theta))      # [l, m, pts]
    cm = np.cos(m[:, None] * phi[None, :])
    sm = np.sin(m[:, None] * phi[None, :])
    uc = np.moveaxis(UC[0, n], 0, -1)
    us = np.moveaxis(US[0, n], 0, -1)
    return -G * np.einsum("lm,lmx->x", N, P * (cm[None] * uc + sm[None] * us))


def solve_polar(r_edges, n_theta, n_phi, lmax, G, rho, tables=None):
    """Full solve on the polar grid: rho[1, n_R, n_theta, n_phi] ->
    Phi[1, n_R, n_theta, n_phi] at the outer interfaces and the angular
    cell midpoints.  Moments by Eqs. (21)-(22) (those of Eqs. 26-27 with
    unit weights), radial sums by Eqs. (19)-(20), synthesis by Eq. (5)."""
    th, ph, w, T, C, S = tables or _polar_tables(n_theta, n_phi, lmax)
    AC, AS = moments(rho, w, T, C, S)
    UC, US = radial_sums(AC, AS, r_edges)
    nR = len(r_edges) - 1
    tc = 0.5 * (th[:-1] + th[1:])
    pc = 0.5 * (ph[:-1] + ph[1:])
    TT, PP = np.meshgrid(tc, pc, indexing="ij")
    tt, pp = TT.ravel(), PP.ravel()
    out = np.zeros((1, nR, n_theta * n_phi))
    for n in range(nR):
        out[0, n] = potential_polar_at(UC, US, G, np.full(tt.shape, n), tt, pp)
    return out.reshape(1, nR, n_theta, n_phi)


def solve_polar_sampled(r_edges, n_theta, n_phi, lmax, G, rho, samples, tables=None,
                        return_moments=False):
    """Phi on the polar grid at selected outputs (p, n, j, k) with p = 0;
    moments and radial sums in full, synthesis only at the samples."""
    th, ph, w, T, C, S = tables or _polar_tables(n_theta, n_phi, lmax)
    AC, AS = moments(rho, w, T, C, S)
    UC, US = radial_sums(AC, AS, r_edges)
    samples = np.asarray(samples)
    tc = 0.5 * (th[:-1] + th[1:])
    pc = 0.5 * (ph[:-1] + ph[1:])
    vals = potential_polar_at(UC, US, G, samples[:, 1], tc[samples[:, 2]], pc[samples[:, 3]])
    if return_moments:
        return vals, (AC, AS)
    return vals
