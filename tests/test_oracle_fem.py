"""Pins of the oracle's discretisation (CPU only).

Each test checks the oracle against something other than itself: closed
forms, invariants, brute force, special cases that reduce to an ODE, and the
observed orders of accuracy the paper prints.
"""
import os

import numpy as np
import pytest
import scipy.optimize

import seird_inputs as si
from oracle import fem, mms, newton, ode

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geo(nx=8):
    xy, tri = si.square_mesh(nx)
    return xy, tri, fem.Geometry(xy, tri)


def test_p1_closed_form_on_structured_mesh():
    """On the right-triangle mesh the P1 stiffness is the 5-point stencil
    and the interior lumped mass is h^2 (textbook closed forms)."""
    nx = 8
    xy, tri, geo = _geo(nx)
    h = 1.0 / nx
    assert np.allclose(geo.area, 0.5 * h * h)
    phi = np.random.default_rng(1).uniform(0.1, 0.9, len(xy))
    # keep N == 1 so that the diffusion coefficient is exactly nu
    u = np.zeros((len(xy), 5))
    u[:, 0] = phi
    u[:, 1] = 1.0 - phi
    nu = (0.3, 0.0, 0.0, 0.0, 0.0)
    dif = fem.diffusion(u, geo, nu)[:, 0]
    P = phi.reshape(nx + 1, nx + 1)
    for j in range(1, nx):
        for i in range(1, nx):
            k = j * (nx + 1) + i
            lap = 4 * P[j, i] - P[j, i - 1] - P[j, i + 1] - P[j - 1, i] - P[j + 1, i]
            assert dif[k] == pytest.approx(0.3 * lap, rel=1e-12, abs=1e-14)
            assert geo.mass[k] == pytest.approx(h * h, rel=1e-14)
    # corners of the two kinds: (0,0) touches 2 triangles, (1,0) one
    assert geo.mass[0] == pytest.approx(2 * 0.5 * h * h / 3)
    assert geo.mass[nx] == pytest.approx(0.5 * h * h / 3)


def test_stiffness_rows_sum_to_zero_and_symmetric():
    """Neumann stiffness: constants are in the kernel; K^T is symmetric."""
    cfg = si.config_realistic(n_base=60, n_ref=1, n_sub=4)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    assert np.all(geo.area > 0)
    assert np.allclose(geo.K.sum(2), 0.0, atol=1e-12)
    assert np.allclose(geo.K, np.transpose(geo.K, (0, 2, 1)))
    u = np.tile([0.5, 0.2, 0.1, 0.1, 0.1], (geo.n, 1))
    assert np.abs(fem.diffusion(u, geo, (1, 1, 1, 1, 1))).max() < 1e-12
    assert geo.mass.sum() == pytest.approx(si.polygon_area(si.star_polygon(1)),
                                           rel=0.05)


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.05, 1.0, (n, 5))
    u[:, 0] += 1.0
    return u


def test_jacobian_matches_central_differences():
    """Brute force: J d equals the central difference of F along random
    directions d (relative 1e-7 at h = 1e-6)."""
    cfg = si.config_realistic(n_base=60, n_ref=1, n_sub=4)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    p = si.Params(**{**si.params_ontario().__dict__, "nu": (0.05, 0.03, 0.02, 0.01, 0.004),
                     "alpha": 0.01, "mu": 0.02})
    u = cfg.u0 * np.random.default_rng(3).uniform(0.5, 1.5, cfg.u0.shape) + 0.1
    up = cfg.u0
    g = np.random.default_rng(4).uniform(0.5, 1.5, geo.n)
    J = fem.jacobian(u, 0.7, geo, p, g)
    rng = np.random.default_rng(5)
    for _ in range(5):
        d = rng.standard_normal(u.shape)
        h = 1e-6
        fd = (fem.residual(u + h * d, up, 0.7, geo, p, g)
              - fem.residual(u - h * d, up, 0.7, geo, p, g)).ravel() / (2 * h)
        an = J @ d.ravel()
        assert np.linalg.norm(fd - an) <= 1e-7 * np.linalg.norm(an)


def test_dense_fd_jacobian_tiny_mesh():
    """Dense finite-difference Jacobian on a 2x2 mesh, entry by entry."""
    xy, tri, geo = _geo(2)
    p = si.params_square()
    p = si.Params(**{**p.__dict__, "nu": (0.2, 0.1, 0.05, 0.3, 0.0)})
    u = _rand_state(geo.n, 7)
    J = fem.jacobian(u, 0.3, geo, p).toarray()
    n5 = 5 * geo.n
    Jfd = np.zeros((n5, n5))
    h = 1e-6
    for k in range(n5):
        d = np.zeros(n5)
        d[k] = h
        Jfd[:, k] = (fem.residual(u + d.reshape(-1, 5), u, 0.3, geo, p)
                     - fem.residual(u - d.reshape(-1, 5), u, 0.3, geo, p)).ravel() / (2 * h)
    assert np.abs(J - Jfd).max() <= 1e-8 * np.abs(J).max()


def test_newton_root_equals_brute_force_root():
    """Tiny mesh: the Newton root equals the root found by a generic
    root finder with its own finite-difference Jacobian (MINPACK hybrd)."""
    xy, tri, geo = _geo(3)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0.02, 0.02, 0.01, 0.02, 0.0)})
    u0 = si.gaussian_bump_state(xy, 0, peak=0.2, width=0.3)
    dt = 0.5
    u1, info = newton.newton_step(u0, dt, geo, p, tol=1e-13)
    sol = scipy.optimize.root(
        lambda x: fem.residual(x.reshape(-1, 5), u0, dt, geo, p).ravel(),
        u0.ravel(), method="hybr", tol=1e-14)
    assert sol.success
    assert np.abs(sol.x.reshape(-1, 5) - u1).max() <= 1e-10 * np.abs(u1).max()
    # quadratic convergence of the exact Jacobian: the last ratio is tiny
    h = info["res_hist"]
    assert len(h) >= 2 and h[-1] < 1e-13


def test_population_conserved_and_nonnegative_small_config():
    """Isolated domain with alpha = mu = 0 conserves sum_i m_i N_i
    (Section 2.1); the right-triangle mesh gives an M-matrix, so the
    densities stay nonnegative."""
    cfg = si.config_small(nx=32)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    u = cfg.u0
    P0 = fem.total_population(u, geo)
    for _ in range(5):
        u, info = newton.newton_step(u, cfg.dt, geo, cfg.params, tol=1e-12)
        assert abs(fem.total_population(u, geo) - P0) <= 1e-12 * P0
        assert u.min() >= -1e-14 * u.max()


def test_zero_diffusion_reduces_to_nodewise_ode():
    """With nu = 0 each node follows backward Euler on the compartmental ODE
    of Appendix B.4 (per-node Newton, independent code path)."""
    xy, tri, geo = _geo(4)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0, 0, 0, 0, 0)})
    u0 = _rand_state(geo.n, 11)
    dt = 0.1
    u = u0.copy()
    for _ in range(5):
        u, _ = newton.newton_step(u, dt, geo, p, tol=1e-14)
    for k in range(0, geo.n, 5):
        ref = ode.backward_euler(u0[k], dt, 5, p)[-1]
        assert np.allclose(u[k], ref, rtol=1e-11, atol=1e-14)


def test_ode_limit_first_order_in_time():
    """Uniform field, zero diffusion: error against a DOP853 reference of the
    ODE decreases with observed order ~1 (Appendix B order table ~1)."""
    xy, tri, geo = _geo(1)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0, 0, 0, 0, 0)})
    y0 = np.array([0.9, 0.0, 0.1, 0.0, 0.0])
    T = 10.0
    ref = ode.reference_solution(y0, T, p)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        u = np.tile(y0, (geo.n, 1))
        for _ in range(int(round(T / dt))):
            u, _ = newton.newton_step(u, dt, geo, p, tol=1e-14)
        errs.append(np.linalg.norm(u[0] - ref) / np.linalg.norm(ref))
    orders = [mms.observed_order(errs[k], errs[k + 1], 2) for k in range(2)]
    assert all(0.95 <= o <= 1.05 for o in orders), orders


def test_picard_and_picard_gs_reach_the_newton_root():
    """Eq. weak_vec_implicit (coupled Picard) and the Appendix A sweep are
    fixed-point iterations for the same discrete root."""
    xy, tri, geo = _geo(8)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0.01, 0.01, 0.005, 0.01, 0.0)})
    u0 = si.gaussian_bump_state(xy, 2, peak=0.05, width=0.2)
    un, _ = newton.newton_step(u0, 0.2, geo, p, tol=1e-13)
    up, _ = newton.picard_step(u0, 0.2, geo, p, tol=1e-14)
    ug, _ = newton.picard_gs_step(u0, 0.2, geo, p, tol=1e-14)
    assert np.abs(up - un).max() <= 1e-11
    assert np.abs(ug - un).max() <= 1e-11


def test_picard_gs_with_vital_dynamics_and_nu_d_reaches_the_newton_root():
    """With births, deaths, a diffusing D and a transmission field, the
    Appendix A sweep (mu on the diagonals, alpha N lagged on the S
    right-hand side) still converges to the coupled Newton root; dropping
    the births from the sweep moves its fixed point off the root."""
    xy, tri, geo = _geo(8)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0.01, 0.012, 0.005, 0.01, 0.004),
                     "alpha": 0.02, "mu": 0.01})
    u0 = si.gaussian_bump_state(xy, 3, peak=0.05, width=0.2)
    g = np.random.default_rng(1).uniform(0.7, 1.3, geo.n)
    un, _ = newton.newton_step(u0, 0.3, geo, p, g, tol=1e-13)
    ug, info = newton.picard_gs_step(u0, 0.3, geo, p, g, tol=1e-14)
    assert np.abs(ug - un).max() <= 1e-11 * np.abs(un).max()
    assert info["eps_hist"][-1] <= 1e-14 and info["its"] >= 3
    p0 = si.Params(**{**p.__dict__, "alpha": 0.0})
    ug0, _ = newton.picard_gs_step(u0, 0.3, geo, p0, g, tol=1e-14)
    assert np.abs(ug0 - un).max() > 1e-6


def _golden_orders():
    out = {}
    with open(os.path.join(GOLDEN, "paper_mms_orders.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = [float(x) for x in v]
    return out


def test_mms_spatial_order_matches_paper():
    """Manufactured solution with homogeneous Neumann data: observed L2
    order in h within the range the paper prints for P1 (+-0.1)."""
    gold = _golden_orders()["spatial"]
    base = si.Params(sigma=1 / 7, gamma_E=1 / 6, gamma_R=1 / 24, gamma_D=1 / 160,
                     A=100.0, beta_I=3.78e-4, beta_E=3.78e-4,
                     nu=(3.94e-4, 3.94e-4, 1e-6, 3.94e-4, 0.0))
    errs = [mms.spatial_error(nx, base) for nx in (8, 16, 32)]
    orders = [mms.observed_order(errs[k], errs[k + 1], 2) for k in range(2)]
    for o in orders:
        assert min(gold) - 0.1 <= o <= max(gold) + 0.1, (orders, errs)


def test_mms_temporal_order_matches_paper():
    gold = _golden_orders()["temporal"]
    p = si.Params(sigma=1 / 7, gamma_E=1 / 6, gamma_R=1 / 24, gamma_D=1 / 160,
                  A=100.0, beta_I=3.78e-4, beta_E=3.78e-4,
                  nu=(3.94e-6, 3.94e-6, 1e-8, 3.94e-6, 0.0))
    uex, f = mms.temporal_case(p)
    xy, tri, geo = _geo(1)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        u = np.tile(uex(0.0), (geo.n, 1))
        for n in range(int(round(5.0 / dt))):
            u, _ = newton.newton_step(u, dt, geo, p, src=np.tile(f((n + 1) * dt), (geo.n, 1)),
                                      tol=1e-14)
        errs.append(mms.rel_l2_error(u, np.tile(uex(5.0), (geo.n, 1)), geo.mass))
    orders = [mms.observed_order(errs[k], errs[k + 1], 2) for k in range(2)]
    for o in orders:
        assert min(gold) - 0.05 <= o <= max(gold) + 0.05, orders


def test_planted_sign_error_is_caught_by_conservation(monkeypatch):
    """A plausible mistake planted in the oracle (wrong sign of the sigma
    term in the infected equation) breaks conservation."""
    cfg = si.config_small(nx=8)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    orig = fem.reaction

    def bad(u, p, g=None):
        r = orig(u, p, g)
        r[:, 2] -= 2 * p.sigma * u[:, 1]
        return r

    monkeypatch.setattr(fem, "reaction", bad)
    u0 = cfg.u0.copy()
    u0[:, 1] = 0.01
    u1, _ = newton.newton_step(u0, cfg.dt, geo, cfg.params, tol=1e-12,
                               linsolve=lambda J, b: np.linalg.lstsq(J.toarray(), b, rcond=None)[0])
    P0 = fem.total_population(u0, geo)
    assert abs(fem.total_population(u1, geo) - P0) > 1e-6 * P0


# ---------------------------------------------------------------------------
# Discretisation and model variants: consistent mass, Neumann flux data,
# the transmission rate's time and space profiles (Section 4.2).
# ---------------------------------------------------------------------------

def test_consistent_mass_closed_form_on_the_square_mesh():
    """Right-triangle mesh of spacing h: an interior row of the consistent
    mass matrix is h^2/2 on the diagonal and h^2/12 for each of its six
    neighbours; every row sums to the lumped mass; M is symmetric."""
    nx = 8
    xy, tri, geo = _geo(nx)
    h = 1.0 / nx
    M = geo.consistent_mass().tocsr()
    assert abs(M - M.T).max() == 0.0
    assert np.allclose(np.asarray(M.sum(1)).ravel(), geo.mass, rtol=1e-14)
    k = 4 * (nx + 1) + 4   # an interior node
    row = M.getrow(k).toarray().ravel()
    assert row[k] == pytest.approx(h * h / 2, rel=1e-13)
    nb = np.nonzero(row)[0]
    assert len(nb) == 7
    for j in nb[nb != k]:
        assert row[j] == pytest.approx(h * h / 12, rel=1e-13)


def test_boundary_flux_integral_closed_forms():
    """The boundary term of nodal flux fields integrates exactly for linear
    fields (divergence theorem on the unit square): a constant flux gives
    zero net outflow, q = (x, y) gives 2 (= div q times the area), and
    q = (x, 0) gives 1."""
    xy, tri, geo = _geo(6)
    q = np.zeros((geo.n, 5, 2))
    q[:, 0, :] = [0.3, -1.2]
    q[:, 1, 0], q[:, 1, 1] = xy[:, 0], xy[:, 1]
    q[:, 2, 0] = xy[:, 0]
    b = geo.boundary_load(q).sum(0)
    assert abs(b[0]) <= 1e-14 and b[1] == pytest.approx(2.0, rel=1e-14) and b[2] == pytest.approx(1.0, rel=1e-14)
    _, nl = geo.boundary_edges()
    assert np.linalg.norm(nl, axis=1).sum() == pytest.approx(4.0, rel=1e-14)


def _mms_params():
    return si.Params(sigma=1 / 7, gamma_E=1 / 6, gamma_R=1 / 24, gamma_D=1 / 160,
                     A=100.0, beta_I=3.78e-4, beta_E=3.78e-4,
                     nu=(3.94e-4, 3.94e-4, 1e-6, 3.94e-4, 0.0))


@pytest.mark.parametrize("mass", ["lumped", "consistent"])
def test_mms_with_neumann_flux_second_order(mass):
    """The paper's 2D manufactured profile with its (time-dependent)
    Neumann data: observed L2 order in h within the paper's printed range
    (+-0.1), with lumped and with consistent mass."""
    gold = _golden_orders()["spatial"]
    p = _mms_params()
    errs = [mms.neumann_spatial_error(nx, p, mass=mass) for nx in (8, 16, 32)]
    orders = [mms.observed_order(errs[k], errs[k + 1], 2) for k in range(2)]
    for o in orders:
        assert min(gold) - 0.1 <= o <= max(gold) + 0.1, (orders, errs)


def test_planted_missing_flux_is_caught_by_the_mms_order():
    """Dropping the boundary flux (the homogeneous-Neumann mistake) leaves
    an error that does not decrease at second order."""
    p = _mms_params()
    errs = [mms.neumann_spatial_error(nx, p, with_flux=False) for nx in (8, 16, 32)]
    orders = [mms.observed_order(errs[k], errs[k + 1], 2) for k in range(2)]
    assert max(orders) < 1.5, (orders, errs)


def test_consistent_mass_jacobian_and_conservation():
    """Consistent mass: the Jacobian agrees with central differences, and
    the total population sum_i m_i N_i is still conserved (the columns of M
    sum to the lumped masses) with alpha = mu = 0 and no flux."""
    xy, tri, geo = _geo(4)
    p = si.Params(**{**si.params_square().__dict__, "nu": (0.02, 0.01, 0.005, 0.02, 0.003)})
    u = _rand_state(geo.n, 5)
    J = fem.jacobian(u, 0.3, geo, p, mass="consistent").toarray()
    n5 = 5 * geo.n
    rng = np.random.default_rng(2)
    for _ in range(5):
        d = rng.standard_normal(n5).reshape(-1, 5)
        h = 1e-6
        fd = (fem.residual(u + h * d, u, 0.3, geo, p, mass="consistent")
              - fem.residual(u - h * d, u, 0.3, geo, p, mass="consistent")).ravel() / (2 * h)
        assert np.abs(J @ d.ravel() - fd).max() <= 1e-8 * np.abs(fd).max()
    u0 = si.gaussian_bump_state(xy, 2, peak=0.05, width=0.2)
    P0 = fem.total_population(u0, geo)
    u1, _ = newton.newton_step(u0, 0.3, geo, p, tol=1e-13, mass="consistent")
    assert abs(fem.total_population(u1, geo) - P0) <= 1e-12 * P0
    assert np.abs(u1 - newton.newton_step(u0, 0.3, geo, p, tol=1e-13)[0]).max() > 1e-8


def test_transmission_profiles_match_the_printed_formulas():
    """Eq. beta_ie: 0.101 before the lockdown, 0.076 at day 130 (half the
    drop), 0.051 long after; Eq. beta_x: the central value mid-domain and
    the regional values far east and far west."""
    f = lambda t: fem.beta_time_factor(t, 0.101, 0.05, 1.0, 130.0)  # noqa: E731
    assert f(0.0) == pytest.approx(0.101, abs=1e-12)
    assert f(130.0) == pytest.approx(0.076, rel=1e-14)
    assert f(400.0) == pytest.approx(0.051, abs=1e-12)
    b = lambda x: fem.beta_regional(x, 1.0, 2.0, 0.5, 3.0, -3.0)  # noqa: E731
    assert b(0.0) == pytest.approx(1.0, abs=1e-6)
    assert b(50.0) == pytest.approx(2.0, abs=1e-12)
    assert b(-50.0) == pytest.approx(0.5, abs=1e-12)
    assert b(3.0) == pytest.approx(1.5, abs=1e-6)
