"""Method of manufactured solutions (oracle verification, Appendix B.1).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The forcing is derived symbolically from the PDE system (Eqs. seird1-5) for
a chosen exact solution, so that d_t u - div(nu(u) grad u) - B(u)u = f.
Observed orders use Eq. MMS_order, p = log(E1/E2) / log(r), with the
relative L2 error of Eq. MMS_error summed over the compartments.

Two manufactured solutions (the paper's amplitudes B = 25 and offsets
A_S..A_D = 500, 300, 200, 100, 80, Allee constant A = 100):

* spatial:  u_c = A_c + B cos(pi x) cos(pi y) (1 + 0.2 t) on the unit
  square -- zero normal derivative on every side, so the homogeneous
  Neumann condition of the weak form holds exactly (the paper's 2D MMS uses
  time-dependent Neumann data instead), and linear in time, so backward
  Euler has no temporal truncation error and the error is purely spatial.
  (A steady solution cannot be used: with alpha = mu = 0 the steady discrete
  operator conserves population and is singular.);
* temporal: u_c = A_c + B sin(0.2 t), spatially uniform (the time
  dependence of the paper's 1D/2D solutions), so the error is purely
  temporal;
* neumann: the paper's own 2D profile (Appendix B.3, Eq. MMS2d,
  B sin(10 x y) + A_c) with the time factor (1 + 0.2 t) in place of the
  phase 0.2 t, so that backward Euler again adds no temporal error, on the
  unit square with the Neumann data of the exact solution.  The flux in the
  weak form's boundary term is nu(u) grad u . n with nu(u) = N nu_bar_c
  (Eq. vec_component1); the paper prints its boundary data without the
  N nu_bar_c factor, and this case uses the flux of the weak form.
"""
from __future__ import annotations

import numpy as np
import sympy as sy

from . import fem

OFFSETS = (500.0, 300.0, 200.0, 100.0, 80.0)
AMP = 25.0


def _pde_forcing(u_exprs, x, y, t, p):
    s, e, i, r, d = u_exprs
    N = s + e + i + r + d
    a = 1 - sy.Float(p.A) / N
    inf = a * (sy.Float(p.beta_I) * s * i + sy.Float(p.beta_E) * s * e)
    reac = [
        sy.Float(p.alpha) * N - inf - sy.Float(p.mu) * s,
        inf - (sy.Float(p.sigma) + sy.Float(p.gamma_E) + sy.Float(p.mu)) * e,
        sy.Float(p.sigma) * e - (sy.Float(p.gamma_R) + sy.Float(p.gamma_D) + sy.Float(p.mu)) * i,
        sy.Float(p.gamma_E) * e + sy.Float(p.gamma_R) * i - sy.Float(p.mu) * r,
        sy.Float(p.gamma_D) * i,
    ]
    f = []
    for c, uc in enumerate(u_exprs):
        nu = sy.Float(p.nu[c])
        div = sy.diff(N * nu * sy.diff(uc, x), x) + sy.diff(N * nu * sy.diff(uc, y), y)
        f.append(sy.diff(uc, t) - div - reac[c])
    return f


def spatial_case(p):
    """Returns (u_exact(xy, t) -> [n,5], f(xy, t) -> [n,5])."""
    x, y, t = sy.symbols("x y t", real=True)
    ue = [sy.Float(A) + sy.Float(AMP) * sy.cos(sy.pi * x) * sy.cos(sy.pi * y)
          * (1 + sy.Float(0.2) * t) for A in OFFSETS]
    f = _pde_forcing(ue, x, y, t, p)
    uf = sy.lambdify((x, y, t), ue, "numpy")
    ff = sy.lambdify((x, y, t), f, "numpy")

    def _stack(v, xy):
        return np.stack([np.broadcast_to(np.asarray(c, dtype=np.float64),
                                         xy[:, 0].shape) for c in v], 1)

    def u_exact(xy, tt):
        return _stack(uf(xy[:, 0], xy[:, 1], tt), xy)

    def forcing(xy, tt):
        return _stack(ff(xy[:, 0], xy[:, 1], tt), xy)

    return u_exact, forcing


def spatial_error(nx, p, dt=0.25, steps=4, mesh=None):
    """Relative L2 error (Eq. MMS_error) at t = dt*steps of backward-Euler
    steps on the nx x nx square mesh, started from the exact nodal values
    and driven by the nodal forcing at t^{n+1}."""
    from . import newton
    import seird_inputs as si
    xy, tri = si.square_mesh(nx) if mesh is None else mesh
    geo = fem.Geometry(xy, tri)
    uex, f = spatial_case(p)
    u = uex(xy, 0.0)
    for n in range(steps):
        u, _ = newton.newton_step(u, dt, geo, p, src=f(xy, (n + 1) * dt),
                                  tol=1e-13)
    return rel_l2_error(u, uex(xy, steps * dt), geo.mass)


def neumann_case(p):
    """Returns (u_exact(xy, t) -> [n,5], f(xy, t) -> [n,5],
    flux(xy, t) -> [n,5,2]) with flux_c = nu_c N grad u_c."""
    x, y, t = sy.symbols("x y t", real=True)
    ue = [sy.Float(A) + sy.Float(AMP) * sy.sin(10 * x * y) * (1 + sy.Float(0.2) * t) for A in OFFSETS]
    f = _pde_forcing(ue, x, y, t, p)
    N = sum(ue)
    q = [[sy.Float(p.nu[c]) * N * sy.diff(ue[c], x), sy.Float(p.nu[c]) * N * sy.diff(ue[c], y)]
         for c in range(5)]
    uf = sy.lambdify((x, y, t), ue, "numpy")
    ff = sy.lambdify((x, y, t), f, "numpy")
    qf = sy.lambdify((x, y, t), q, "numpy")

    def _stack(v, xy):
        return np.stack([np.broadcast_to(np.asarray(c, dtype=np.float64), xy[:, 0].shape) for c in v], 1)

    def u_exact(xy, tt):
        return _stack(uf(xy[:, 0], xy[:, 1], tt), xy)

    def forcing(xy, tt):
        return _stack(ff(xy[:, 0], xy[:, 1], tt), xy)

    def flux(xy, tt):
        v = qf(xy[:, 0], xy[:, 1], tt)
        return np.stack([_stack(comp, xy) for comp in v], 1)  # [n, 5, 2]

    return u_exact, forcing, flux


def neumann_spatial_error(nx, p, dt=0.25, steps=4, mass="lumped", with_flux=True, mesh=None):
    """Relative L2 error (Eq. MMS_error) at t = dt*steps for the Neumann
    case on the nx x nx square mesh (flux data and forcing at t^{n+1})."""
    from . import newton
    import seird_inputs as si
    xy, tri = si.square_mesh(nx) if mesh is None else mesh
    geo = fem.Geometry(xy, tri)
    uex, f, q = neumann_case(p)
    u = uex(xy, 0.0)
    for n in range(steps):
        tn = (n + 1) * dt
        u, _ = newton.newton_step(u, dt, geo, p, src=f(xy, tn), tol=1e-13, mass=mass,
                                  neumann=q(xy, tn) if with_flux else None)
    return rel_l2_error(u, uex(xy, steps * dt), geo.mass)


def temporal_case(p):
    """Returns (u_exact(t) -> [5], f(t) -> [5]) for the uniform solution."""
    x, y, t = sy.symbols("x y t", real=True)
    ue = [sy.Float(A) + sy.Float(AMP) * sy.sin(sy.Float(0.2) * t) for A in OFFSETS]
    f = _pde_forcing(ue, x, y, t, p)
    uf = sy.lambdify(t, ue, "numpy")
    ff = sy.lambdify(t, f, "numpy")
    return (lambda tt: np.array(uf(tt), dtype=np.float64),
            lambda tt: np.array(ff(tt), dtype=np.float64))


def rel_l2_error(u_h, u_ex, mass):
    """Eq. MMS_error per compartment (mass-weighted discrete L2 norm),
    summed over the five compartments."""
    num = np.sqrt((mass[:, None] * (u_h - u_ex) ** 2).sum(0))
    den = np.sqrt((mass[:, None] * u_ex ** 2).sum(0))
    return float((num / den).sum())


def observed_order(E1, E2, r):
    """Eq. MMS_order."""
    return float(np.log(E1 / E2) / np.log(r))
