"""Pins of the oracle's 22-compartment model (Appendix C) against what the
equations and the mathematics fix: conservation of the total population,
the affine split of every reaction term, the zero-diffusion limit against
an independent backward-Euler ODE solve, a closed-form special case, and the
Picard-Gauss-Seidel root against the residual."""
import numpy as np
import pytest
import scipy.optimize as so

import seird_inputs as si
from oracle import fem, model22 as m22


def _state(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (n, m22.NC22))


def test_compartment_lists_agree_with_the_inputs_module():
    assert m22.NAMES == si.COMPARTMENTS22
    assert m22.DIFFUSING == si.DIFFUSING22


def test_reactions_conserve_the_total_population():
    """Every flow of Appendix C leaves one compartment and enters another
    (deaths enter D), so the reaction terms sum to zero at any state."""
    p = si.Params22()
    u = _state(50, 1)
    R = m22.reaction22(u, p)
    assert np.abs(R.sum(1)).max() <= 1e-15 * np.abs(R).max() * m22.NC22


def test_planted_reaction_mistakes_break_conservation(monkeypatch):
    """A dropped term or a wrong split factor anywhere shows up in the sum."""
    p = si.Params22()
    u = _state(20, 2)
    base = m22.reaction22
    for k in range(m22.NC22):
        def bad(uu, pp, k=k):
            R = base(uu, pp)
            R[..., k] *= 1.001
            return R
        monkeypatch.setattr(m22, "reaction22", bad)
        assert np.abs(m22.reaction22(u, p).sum(1)).max() > 1e-8
    monkeypatch.setattr(m22, "reaction22", base)
    # a wrong factor inside one flow (sigma_S <-> 1 - sigma_S in C)
    q = si.Params22(sigma_S=0.3)
    R = base(u, q)
    c = {nm: u[:, k] for k, nm in enumerate(m22.NAMES)}
    R[:, m22.IX["C"]] = (1 - q.sigma_A) * (1 - q.sigma_S) * q.gamma_P * c["A"] - q.gamma_S1 * c["C"]
    assert np.abs(R.sum(1)).max() > 1e-8


def test_split_reproduces_every_reaction_term():
    p = si.Params22()
    u = _state(30, 3)
    R = m22.reaction22(u, p)
    for k in range(m22.NC22):
        s, d = m22.split22(k, u, p)
        assert np.allclose(s - d * u[:, k], R[:, k], rtol=1e-13, atol=1e-16), m22.NAMES[k]
        # s and d do not depend on u_k
        v = u.copy()
        v[:, k] *= 3.0
        s2, d2 = m22.split22(k, v, p)
        assert np.array_equal(s, s2) and np.array_equal(d, d2), m22.NAMES[k]


def _ode_step(y, dt, p):
    """Backward Euler of the 22 ODEs at one point, y+ - y - dt R(y+) = 0,
    solved by scipy's hybrid root finder (independent of the sweeps)."""
    f = lambda z: z - y - dt * m22.reaction22(z[None, :], p)[0]
    z = so.fsolve(f, y, xtol=1e-13)
    assert np.abs(f(z)).max() <= 1e-15 * np.abs(y).max() * 10
    return z


def test_zero_diffusion_uniform_state_follows_the_ode():
    p = si.Params22(nu=(0.0,) * 10)
    xy, tri = si.square_mesh(6)
    geo = fem.Geometry(xy, tri)
    y = si.state22(np.array([[0.5, 0.5]]), 0, peak=0.05, width=1.0)[0]
    u = np.tile(y, (geo.n, 1))
    for _ in range(3):
        u, _ = m22.picard_gs_step22(u, 1.0, geo, p, tol=1e-14)
        y = _ode_step(y, 1.0, p)
    assert np.abs(u - y[None, :]).max() <= 1e-11 * np.abs(y).max()


def test_vaccination_exchange_has_its_closed_form():
    """With no infection (only S and V populated) the step is the 2x2 linear
    backward-Euler system of S' = -g_V S + g_T V, V' = g_V S - g_T V."""
    p = si.Params22(nu=(0.0,) * 10)
    xy, tri = si.square_mesh(4)
    geo = fem.Geometry(xy, tri)
    u0 = np.zeros((geo.n, m22.NC22))
    u0[:, m22.IX["S"]] = 0.8
    u0[:, m22.IX["V"]] = 0.2
    dt = 5.0
    u, _ = m22.picard_gs_step22(u0, dt, geo, p, tol=1e-15)
    A = np.array([[1 + dt * p.gamma_V, -dt * p.gamma_T], [-dt * p.gamma_V, 1 + dt * p.gamma_T]])
    sv = np.linalg.solve(A, [0.8, 0.2])
    assert np.allclose(u[:, m22.IX["S"]], sv[0], rtol=1e-13)
    assert np.allclose(u[:, m22.IX["V"]], sv[1], rtol=1e-13)
    others = [k for k in range(m22.NC22) if m22.NAMES[k] not in ("S", "V")]
    assert np.abs(u[:, others]).max() == 0.0


@pytest.fixture(scope="module")
def spread():
    xy, tri = si.square_mesh(12)
    geo = fem.Geometry(xy, tri)
    p = si.Params22(nu=(2e-2, 2e-2, 2e-2, 1e-2, 1e-2, 5e-3, 2e-3, 5e-3, 2e-2, 2e-2))
    u0 = si.state22(xy, 4, peak=0.05, width=0.15)
    return geo, p, u0


def test_sweeps_reach_a_root_of_the_coupled_residual(spread):
    geo, p, u0 = spread
    u, hist = m22.picard_gs_step22(u0, 1.0, geo, p, tol=1e-13)
    F = m22.residual22(u, u0, 1.0, geo, p)
    assert np.linalg.norm(F) <= 1e-11 * np.linalg.norm(geo.mass[:, None] * u0)
    assert hist[-1] <= 1e-13 and len(hist) > 3
    # total population conserved (stiffness columns and reactions sum to 0)
    tot0 = (geo.mass[:, None] * u0).sum()
    tot1 = (geo.mass[:, None] * u).sum()
    assert abs(tot1 - tot0) <= 1e-11 * tot0
    assert u.min() >= -1e-14


def test_diffusion_of_the_nodal_compartments_is_off(spread):
    """Only the ten diffusing compartments feel the stiffness term: with all
    rates zero a bump in E spreads while the same bump in Q stays put."""
    geo, p, u0 = spread
    zero = si.Params22(**{f: 0.0 for f in si.Params22.__dataclass_fields__ if f != "nu"}, nu=p.nu)
    u = np.zeros_like(u0)
    bump = u0[:, m22.IX["E"]] + u0[:, m22.IX["A"]]
    u[:, m22.IX["E"]] = bump
    u[:, m22.IX["Q"]] = bump
    v, _ = m22.picard_gs_step22(u, 1.0, geo, zero, tol=1e-14)
    assert np.allclose(v[:, m22.IX["Q"]], bump, rtol=1e-15, atol=0)
    assert np.abs(v[:, m22.IX["E"]] - bump).max() > 1e-4 * bump.max()
    K = m22.stiffness(geo)
    lhs = geo.mass * (v[:, m22.IX["E"]] - bump) + p.nu[2] * (K @ v[:, m22.IX["E"]])
    assert np.abs(lhs).max() <= 1e-13 * bump.max()
