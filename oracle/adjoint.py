"""Discrete adjoint of a case-count misfit (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The forward model is the sequence of backward-Euler residual equations
F^n(u^n, u^{n-1}; theta) = 0, n = 1..N (``fem.residual``), with parameters
theta = (g, nu): the per-node transmission multiplier g (beta_I and beta_E
at node j are scaled by g_j, the product form of Eq. beta_ie) and the five
diffusion coefficients nu_bar_c (Eq. vec_component1).  The observation is the
infected count of every region r at every step, c_r^n = sum_{j in r} m_j
i_j^n, and the misfit J = sum_n sum_r (c_r^n - target_r^n)^2.

With dF^{n+1}/du^n = -M (lumped mass on every compartment), the adjoint
states solve, for n = N down to 1,

    (dF^n/du^n)^T lam^n = dJ/du^n + M lam^{n+1},      lam^{N+1} = 0,

and the gradient is dJ/dtheta = - sum_n (dF^n/dtheta)^T lam^n.  The only
theta-dependent terms of F are
    dF_{S,j}/dg_j = + dt m_j a_j (beta_I i_j + beta_E e_j) s_j
    dF_{E,j}/dg_j = - dt m_j a_j (beta_I i_j + beta_E e_j) s_j
    dF_{c,i}/dnu_c = dt sum_{T ni i} Nbar_T sum_{k in T} K^T_ik u_{c,k}
(a_j the Allee factor), all evaluated at u^n.

The sweep keeps every state (no checkpointing) and solves with a sparse LU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, newton

NC = 5
I_COMP = 2


def region_counts(u, mass, region, n_regions):
    """c_r = sum_{j in r} m_j i_j; nodes with region < 0 are unobserved."""
    c = np.zeros(n_regions)
    sel = region >= 0
    np.add.at(c, region[sel], mass[sel] * u[sel, I_COMP])
    return c


def forward(u0, steps, dt, geo, p, g, region, n_regions, tol=1e-13):
    """All states u^0..u^N and the counts [N, n_regions]."""
    states = [np.array(u0, dtype=np.float64)]
    counts = []
    u = states[0]
    for _ in range(steps):
        u, _ = newton.newton_step(u, dt, geo, p, g, tol=tol)
        states.append(u)
        counts.append(region_counts(u, geo.mass, region, n_regions))
    return states, np.array(counts)


def misfit(counts, target):
    return float(((counts - target) ** 2).sum())


def adjoint_gradient(states, dt, geo, p, g, region, n_regions, grad_counts):
    """Gradient of a loss whose derivative with respect to the counts is
    ``grad_counts`` [N, n_regions] (2 (c - target) for the squared misfit).
    Returns (grad_g [n], grad_nu [5])."""
    n = geo.n
    N = len(states) - 1
    gg = np.ones(n) if g is None else np.asarray(g, dtype=np.float64)
    m = geo.mass
    grad_g = np.zeros(n)
    grad_nu = np.zeros(NC)
    lam_next = np.zeros((n, NC))
    sel = region >= 0
    for k in range(N, 0, -1):
        u = states[k]
        J = fem.jacobian(u, dt, geo, p, gg)
        rhs = m[:, None] * lam_next
        rhs[sel, I_COMP] += grad_counts[k - 1][region[sel]] * m[sel]
        lam = spla.splu(J.T.tocsc()).solve(rhs.ravel()).reshape(n, NC)
        s, e, i = u[:, 0], u[:, 1], u[:, 2]
        N_ = u.sum(1)
        a = 1.0 - p.A / N_
        dFS_dg = dt * m * a * (p.beta_I * i + p.beta_E * e) * s
        grad_g -= lam[:, 0] * dFS_dg - lam[:, 1] * dFS_dg
        D = fem.diffusion(u, geo, np.ones(NC))     # diffusion with nu_c = 1
        grad_nu -= dt * (lam * D).sum(0)
        lam_next = lam
    return grad_g, grad_nu
