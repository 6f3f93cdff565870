"""CPU checks of the ellipsoid validation inputs: the semi-analytic potential
against closed forms and direct quadrature, and the cell-averaged density
against the ellipsoid's volume."""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from paper_1806_04593_amd import validation as V


def test_sphere_limit_of_the_ellipsoid_potential():
    R, G, rho0 = 0.7, 1.3, 2.0
    r = np.array([0.0, 0.1, 0.35, 0.69, 0.71, 1.0, 3.0])
    d = np.array([1.0, 2.0, -1.5])
    d /= np.linalg.norm(d)
    x = r[:, None] * d[None]
    got = V.ellipsoid_potential(x[:, 0], x[:, 1], x[:, 2], R, R, R, G, rho0)
    M = 4.0 / 3.0 * math.pi * R ** 3 * rho0
    ex = np.where(r <= R, -2.0 * math.pi * G * rho0 * (R * R - r * r / 3.0), -G * M / np.maximum(r, 1e-300))
    np.testing.assert_allclose(got, ex, rtol=1e-13)


@pytest.mark.parametrize("pt", [(0.1, 0.2, 0.3), (0.4, -0.5, 0.2), (1.2, 0.3, -0.4), (0.0, 0.0, 2.5)])
def test_ellipsoid_potential_against_quadrature(pt):
    """The four integrals of Sect. 5 by adaptive quadrature (u -> t = 1/(1+u)
    maps the infinite range to (0, 1])."""
    a, b, c = V.axes(1.0)
    x, y, z = pt

    def f(u):
        return x * x / (a * a + u) + y * y / (b * b + u) + z * z / (c * c + u) - 1.0
    u0 = 0.0
    if f(0.0) > 0:
        from scipy import optimize
        hi = 1.0
        while f(hi) > 0:
            hi *= 2
        u0 = optimize.brentq(f, 0.0, hi, xtol=1e-15, rtol=1e-15)

    def integral(pa, pb, pc):
        def g(t):
            u = u0 + (1.0 - t) / t
            return ((a * a + u) ** pa * (b * b + u) ** pb * (c * c + u) ** pc) ** -0.5 / (t * t)
        return integrate.quad(g, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=200)[0]
    A, B, C, D = integral(3, 1, 1), integral(1, 3, 1), integral(1, 1, 3), integral(1, 1, 1)
    ex = math.pi * a * b * c * (A * x * x + B * y * y + C * z * z - D)
    got = V.ellipsoid_potential(x, y, z, a, b, c)
    assert abs(got - ex) <= 1e-12 * abs(ex)


def test_potential_continuous_across_the_surface():
    a, b, c = V.axes(1.0)
    d = np.array([0.3, -0.8, 0.5])
    s = math.sqrt((d[0] / a) ** 2 + (d[1] / b) ** 2 + (d[2] / c) ** 2)
    t = np.array([1.0 - 1e-9, 1.0 + 1e-9]) / s
    v = V.ellipsoid_potential(t * d[0], t * d[1], t * d[2], a, b, c)
    assert abs(v[0] - v[1]) < 1e-8 * abs(v[0])


@pytest.mark.parametrize("kind", ["yinyang", "polar"])
def test_volume_fraction_recovers_the_volume(kind):
    d = V._grid_desc(kind, 40, 6.0, 0)
    rho = V.volume_fraction(d, sub=4)
    assert rho.min() >= 0.0 and rho.max() <= 1.0
    r = d["r_edges"]
    th, ph = V._edges(d)
    om = O.solid_angles(th, ph)
    w = np.ones_like(om) if kind == "polar" else O.overlap_weights(th, ph, d["delta_theta"], d["delta_phi"])
    vol = ((r[1:] ** 3 - r[:-1] ** 3) / 3.0)[None, :, None, None] * (om * w)[None, None]
    a, b, c = V.axes(1.0)
    mass = float(np.sum(rho * vol))
    assert abs(mass - 4.0 / 3.0 * math.pi * a * b * c) < 2e-3 * mass
