"""Nonlinear solvers for one backward-Euler step (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

* ``newton_step`` -- fully coupled Newton on the residual of ``fem.residual``
  (the alternative the paper names for strongly coupled systems, Section
  2.2), started from u^n, stopped on the scaled residual
  ||F(u^k)||_2 <= tol * ||M_L u^n||_2; the Picard-style update size
  epsilon of Eq. picardtol is reported.
* ``picard_step`` -- the coupled Picard linearisation of Eq.
  weak_vec_implicit (coefficients nu(u) and B(u) lagged at iterate k).
* ``picard_gs_step`` -- the decoupled per-compartment Picard sweep of
  Appendix A (S, E, I, R, D in turn, each using the compartments already
  updated in the sweep, with N and the Allee factor lagged).

All three reach the same discrete root; only the iteration differs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem

NC = 5


class NotConverged(RuntimeError):
    pass


def direct_solve(J, b):
    if J.shape[0] <= 2000:
        return np.linalg.solve(J.toarray(), b)
    return spla.splu(J.tocsc()).solve(b)


def newton_step(u_prev, dt, geo, p, g=None, src=None, tol=1e-10, max_it=20,
                linsolve=None, mass="lumped", neumann=None):
    """One implicit step by Newton's method.  Returns (u_next, info) where
    info holds the Newton count, the scaled residual history and epsilon.
    ``mass`` and ``neumann`` select the discretisation variant (see
    fem.residual); the stopping scale stays ||M_L u^n||."""
    linsolve = direct_solve if linsolve is None else linsolve
    u = np.array(u_prev, dtype=np.float64, copy=True)
    scale = np.linalg.norm(geo.mass[:, None] * u_prev)
    unorm = np.linalg.norm(u_prev)
    hist, eps_hist, lin_info = [], [], []
    for k in range(max_it + 1):
        F = fem.residual(u, u_prev, dt, geo, p, g, src, mass=mass, neumann=neumann)
        fn = np.linalg.norm(F)
        hist.append(fn / scale)
        if not np.isfinite(fn):
            raise NotConverged("nonfinite residual")
        if fn <= tol * scale:
            return u, dict(newton_its=k, res_hist=hist, eps_hist=eps_hist,
                           lin=lin_info)
        if k == max_it:
            break
        J = fem.jacobian(u, dt, geo, p, g, mass=mass)
        out = linsolve(J, -F.ravel())
        if isinstance(out, tuple):
            delta, li = out
            lin_info.append(li)
        else:
            delta = out
        delta = delta.reshape(-1, NC)
        u = u + delta
        eps_hist.append(np.linalg.norm(delta) / unorm)
    raise NotConverged(f"Newton did not reach {tol} in {max_it} its: {hist}")


def _stiffness(geo, coef_T):
    """Scalar P1 matrix sum_T coef_T K^T (n x n)."""
    tri = geo.tri
    r = np.repeat(tri, 3, axis=1).ravel()
    c = np.tile(tri, (1, 3)).ravel()
    v = (coef_T[:, None, None] * geo.K).reshape(-1)
    return sp.coo_matrix((v, (r, c)), shape=(geo.n, geo.n)).tocsr()


def reaction_matrix(u, p, g=None):
    """B(u) of Eq. vec_component2 per node, [n,5,5], so that B(u) u is the
    reaction term."""
    s, e, i, r, d = u.T
    N = s + e + i + r + d
    gg = np.ones_like(s) if g is None else np.broadcast_to(g, s.shape)
    a = 1.0 - p.A / N
    B = np.zeros((len(s), NC, NC))
    B[:, 0, 0] = p.alpha - p.mu - a * gg * p.beta_E * e - a * gg * p.beta_I * i
    B[:, 0, 1:] = p.alpha
    B[:, 1, 0] = a * gg * p.beta_I * i
    B[:, 1, 1] = a * gg * p.beta_E * s - p.mu - p.sigma - p.gamma_E
    B[:, 2, 1] = p.sigma
    B[:, 2, 2] = -p.gamma_R - p.gamma_D - p.mu
    B[:, 3, 1] = p.gamma_E
    B[:, 3, 2] = p.gamma_R
    B[:, 3, 3] = -p.mu
    B[:, 4, 2] = p.gamma_D
    return B


def picard_step(u_prev, dt, geo, p, g=None, tol=1e-12, max_it=200):
    """Coupled Picard iteration of Eq. weak_vec_implicit: solve
    M u^{k+1} + dt K(N^k) u^{k+1} - dt M B(u^k) u^{k+1} = M u^n, stop on
    epsilon of Eq. picardtol."""
    n = geo.n
    u = u_prev.copy()
    unorm = np.linalg.norm(u_prev)
    m = geo.mass
    rhs = (m[:, None] * u_prev).ravel()
    for k in range(1, max_it + 1):
        Nbar = u.sum(1)[geo.tri].mean(1)
        Kn = _stiffness(geo, Nbar)
        blocks = []
        B = reaction_matrix(u, p, g)
        Mb = sp.block_diag([m[i] * (np.eye(NC) - dt * B[i]) for i in range(n)],
                           format="csr")
        Kfull = sp.kron(Kn, sp.diags(dt * np.asarray(p.nu)), format="csr")
        A = (Mb + Kfull).tocsc()
        un = spla.spsolve(A, rhs).reshape(-1, NC)
        eps = np.linalg.norm(un - u) / unorm
        u = un
        if eps <= tol:
            return u, dict(its=k, eps=eps)
    raise NotConverged("Picard")


def picard_gs_step(u_prev, dt, geo, p, g=None, tol=1e-12, max_it=500):
    """Decoupled Picard sweep of Appendix A, lumped mass.  Appendix A drops
    the vital dynamics (alpha = mu = 0); with them, mu is a loss on every
    compartment's diagonal except D's and the births alpha N enter the
    susceptible right-hand side with N lagged, which leaves the fixed point
    equal to the root of the coupled residual (Eq. vec_component2)."""
    n = geo.n
    m = geo.mass
    gg = np.ones(n) if g is None else g
    nu = np.asarray(p.nu)
    u = u_prev.copy()
    unorm = np.linalg.norm(u_prev)
    sn, en, in_, rn, dn = u_prev.T
    Mdiag = sp.diags(m)
    eps_hist = []
    for k in range(1, max_it + 1):
        s, e, i, r, d = u.T.copy()
        N = s + e + i + r + d
        a = 1.0 - p.A / N
        Kn = _stiffness(geo, N[geo.tri].mean(1))
        # susceptible
        A = Mdiag + sp.diags(dt * m * (a * gg * (p.beta_I * i + p.beta_E * e) + p.mu)) + dt * nu[0] * Kn
        s1 = spla.spsolve(A.tocsc(), m * sn + dt * m * p.alpha * N)
        # exposed
        A = Mdiag - sp.diags(dt * m * a * gg * p.beta_E * s1) + \
            sp.diags(dt * m * (p.sigma + p.gamma_E + p.mu) * np.ones(n)) + dt * nu[1] * Kn
        e1 = spla.spsolve(A.tocsc(), m * en + dt * m * a * gg * p.beta_I * s1 * i)
        # infected
        A = Mdiag + sp.diags(dt * m * (p.gamma_D + p.gamma_R + p.mu) * np.ones(n)) + dt * nu[2] * Kn
        i1 = spla.spsolve(A.tocsc(), m * in_ + dt * m * p.sigma * e1)
        # recovered
        A = Mdiag + sp.diags(dt * m * p.mu * np.ones(n)) + dt * nu[3] * Kn
        r1 = spla.spsolve(A.tocsc(), m * rn + dt * m * (p.gamma_R * i1 + p.gamma_E * e1))
        # deceased (no diffusion unless nu_D != 0)
        A = Mdiag + dt * nu[4] * Kn
        d1 = spla.spsolve(A.tocsc(), m * dn + dt * m * p.gamma_D * i1)
        un = np.stack([s1, e1, i1, r1, d1], 1)
        eps = np.linalg.norm(un - u) / unorm
        eps_hist.append(eps)
        u = un
        if eps <= tol:
            return u, dict(its=k, eps=eps, eps_hist=eps_hist)
    raise NotConverged("Picard-GS")
