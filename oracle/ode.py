"""ODE limit of the SEIRD model (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Appendix B.4 compares the PDE with vanishing diffusion and a uniform field
against the compartmental ODE.  In density units (the paper's ODE is written
for proportions with the factor (1 - A); its consistent density form uses
1 - A/N) the ODE is

  s' = -(1-A/N) beta_I s i - (1-A/N) beta_E s e
  e' =  (1-A/N) beta_I s i + (1-A/N) beta_E s e - sigma e - gamma_E e
  i' =  sigma e - (gamma_R + gamma_D) i
  r' =  gamma_E e + gamma_R i
  d' =  gamma_D i

(alpha = mu = 0, as in the paper's studies).
"""
from __future__ import annotations

import numpy as np


def ode_rhs(y, p, g=1.0):
    s, e, i, r, d = y
    N = s + e + i + r + d
    a = 1.0 - p.A / N
    inf = a * g * (p.beta_I * s * i + p.beta_E * s * e)
    return np.array([
        -inf,
        inf - p.sigma * e - p.gamma_E * e,
        p.sigma * e - (p.gamma_R + p.gamma_D) * i,
        p.gamma_E * e + p.gamma_R * i,
        p.gamma_D * i,
    ])


def ode_jac(y, p, g=1.0, h=1e-7):
    """Central finite-difference Jacobian of ``ode_rhs`` (used only inside
    the scalar Newton of ``backward_euler``)."""
    J = np.zeros((5, 5))
    for k in range(5):
        dy = np.zeros(5)
        dy[k] = h * max(1.0, abs(y[k]))
        J[:, k] = (ode_rhs(y + dy, p, g) - ode_rhs(y - dy, p, g)) / (2 * dy[k])
    return J


def backward_euler(y0, dt, steps, p, g=1.0, tol=1e-14):
    """Backward Euler for the ODE above with a per-step Newton iteration."""
    y = np.array(y0, dtype=np.float64)
    out = [y.copy()]
    for _ in range(steps):
        yn = y.copy()
        x = y.copy()
        for _k in range(50):
            G = x - yn - dt * ode_rhs(x, p, g)
            if np.linalg.norm(G) <= tol * max(1.0, np.linalg.norm(yn)):
                break
            Jg = np.eye(5) - dt * ode_jac(x, p, g)
            x = x - np.linalg.solve(Jg, G)
        y = x
        out.append(y.copy())
    return np.array(out)


def reference_solution(y0, t_end, p, g=1.0, rtol=1e-12, atol=1e-14):
    """High-accuracy integration (DOP853) of the ODE."""
    from scipy.integrate import solve_ivp
    sol = solve_ivp(lambda t, y: ode_rhs(y, p, g), (0.0, t_end), y0,
                    method="DOP853", rtol=rtol, atol=atol)
    return sol.y[:, -1]
