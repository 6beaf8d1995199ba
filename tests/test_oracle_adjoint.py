"""Pins of the oracle's discrete adjoint (CPU only): central finite
differences of the misfit in random parameter directions, and the Taylor
remainder of a first-order expansion."""
import numpy as np
import pytest

import seird_inputs as si
from oracle import adjoint, fem


def _setup(nx=6, steps=4):
    xy, tri = si.square_mesh(nx)
    geo = fem.Geometry(xy, tri)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0.02, 0.015, 0.01, 0.02, 0.005)})
    u0 = si.gaussian_bump_state(xy, 3, peak=0.05, width=0.25)
    rng = np.random.default_rng(0)
    g = rng.uniform(0.8, 1.2, geo.n)
    region = (xy[:, 0] > 0.5).astype(np.int32) + 2 * (xy[:, 1] > 0.5).astype(np.int32)
    region[::7] = -1  # some unobserved nodes
    return xy, tri, geo, p, u0, g, region, 4, steps


def _J(u0, steps, dt, geo, p, g, region, nreg, target):
    _, c = adjoint.forward(u0, steps, dt, geo, p, g, region, nreg, tol=1e-14)
    return adjoint.misfit(c, target)


def test_adjoint_gradient_matches_central_differences():
    xy, tri, geo, p, u0, g, region, nreg, steps = _setup()
    dt = 0.5
    states, c = adjoint.forward(u0, steps, dt, geo, p, g, region, nreg, tol=1e-14)
    target = c * 0.9 + 1e-4
    gg, gnu = adjoint.adjoint_gradient(states, dt, geo, p, g, region, nreg, 2 * (c - target))
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(geo.n)
        d /= np.abs(d).max()
        Jp = _J(u0, steps, dt, geo, p, g + h * d, region, nreg, target)
        Jm = _J(u0, steps, dt, geo, p, g - h * d, region, nreg, target)
        fd = (Jp - Jm) / (2 * h)
        assert fd == pytest.approx(gg @ d, rel=1e-5)
    for c in range(5):
        dn = np.zeros(5)
        dn[c] = 1.0
        hc = 1e-4 * p.nu[c]  # central differences: O(hc^2) truncation, roundoff-safe
        pp = si.Params(**{**p.__dict__, "nu": tuple(np.array(p.nu) + hc * dn)})
        pm = si.Params(**{**p.__dict__, "nu": tuple(np.array(p.nu) - hc * dn)})
        fd = (_J(u0, steps, dt, geo, pp, g, region, nreg, target)
              - _J(u0, steps, dt, geo, pm, g, region, nreg, target)) / (2 * hc)
        assert fd == pytest.approx(gnu[c], rel=1e-5, abs=1e-12 * abs(gnu).max())


def test_taylor_remainder_is_second_order():
    """|J(g + h d) - J(g) - h grad.d| = O(h^2)."""
    xy, tri, geo, p, u0, g, region, nreg, steps = _setup(nx=5, steps=3)
    dt = 0.5
    states, c = adjoint.forward(u0, steps, dt, geo, p, g, region, nreg, tol=1e-14)
    target = c * 1.1
    gg, _ = adjoint.adjoint_gradient(states, dt, geo, p, g, region, nreg, 2 * (c - target))
    J0 = adjoint.misfit(c, target)
    d = np.random.default_rng(2).standard_normal(geo.n)
    rem = []
    for h in (1e-2, 5e-3, 2.5e-3):
        Jh = _J(u0, steps, dt, geo, p, g + h * d, region, nreg, target)
        rem.append(abs(Jh - J0 - h * (gg @ d)))
    o1 = np.log(rem[0] / rem[1]) / np.log(2)
    o2 = np.log(rem[1] / rem[2]) / np.log(2)
    assert 1.8 < o1 < 2.2 and 1.8 < o2 < 2.2, (rem, o1, o2)
