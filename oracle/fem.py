"""Spatial discretisation of the SEIRD system on P1 triangles (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The discrete equations follow the weak form (Eq. weakform) with homogeneous
Neumann data (Section 2.2: an isolated domain), P1 elements (Section 2.2,
"triangular elements with linear interpolation functions") and backward
Euler in time (Eq. timediscrete).  Readings where the paper is silent:

* mass and reaction terms use the lumped (nodal) mass m_i = sum_{T ni i}|T|/3;
* the diffusion coefficient nu(u) = N diag(nu_bar) (Eq. vec_component1) is
  P1 because N = s+e+i+r+d (Eq. N, deceased included) is P1, so
  int_T N grad(phi_i).grad(phi_j) = mean_T(N) |T| grad(phi_i).grad(phi_j)
  exactly;
* the spatial transmission field g (default 1) multiplies beta_I and beta_E
  at each node, as the product form of Eq. beta_ie does.

Unknown numbering: node-major, unknown 5*node + c with c = S, E, I, R, D.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

NC = 5


class Geometry:
    """Element areas, constant P1 gradients, element stiffness K^T and the
    lumped mass of a triangle mesh."""

    def __init__(self, xy: np.ndarray, tri: np.ndarray):
        self.xy = np.asarray(xy, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        self.n = len(self.xy)
        p = self.xy[self.tri]                    # [nt, 3, 2]
        x, y = p[..., 0], p[..., 1]
        # twice the signed area
        det = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - \
              (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
        self.area = 0.5 * det
        # grad phi_k = (y_{k+1} - y_{k+2}, x_{k+2} - x_{k+1}) / (2|T|)
        g = np.empty(p.shape)
        for k in range(3):
            k1, k2 = (k + 1) % 3, (k + 2) % 3
            g[:, k, 0] = (y[:, k1] - y[:, k2]) / det
            g[:, k, 1] = (x[:, k2] - x[:, k1]) / det
        self.grad = g
        # K^T_kl = |T| grad phi_k . grad phi_l
        self.K = self.area[:, None, None] * np.einsum("tkd,tld->tkl", g, g)
        m = np.zeros(self.n)
        np.add.at(m, self.tri.ravel(), np.repeat(self.area / 3.0, 3))
        self.mass = m

    def consistent_mass(self) -> sp.csr_matrix:
        """Consistent P1 mass matrix M_ij = int phi_i phi_j, assembled from
        the element matrices |T|/12 (1 + delta_kl)."""
        tri = self.tri
        Me = (np.ones((3, 3)) + np.eye(3))[None, :, :] * (self.area / 12.0)[:, None, None]
        r = np.repeat(tri, 3, axis=1).ravel()
        c = np.tile(tri, (1, 3)).ravel()
        return sp.coo_matrix((Me.reshape(-1), (r, c)), shape=(self.n, self.n)).tocsr()

    def boundary_edges(self):
        """Edges that belong to exactly one triangle: (edges [nb, 2], outward
        normals scaled by the edge lengths [nb, 2]).  The normal points away
        from the triangle's third vertex."""
        tri = self.tri
        e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
        opp = np.concatenate([tri[:, 2], tri[:, 0], tri[:, 1]])
        key = np.sort(e, axis=1)
        _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
        keep = cnt[inv.ravel()] == 1
        b, o = e[keep], opp[keep]
        d = self.xy[b[:, 1]] - self.xy[b[:, 0]]
        nl = np.stack([d[:, 1], -d[:, 0]], 1)        # |nl| = edge length
        away = ((self.xy[b[:, 0]] - self.xy[o]) * nl).sum(1) < 0
        nl[away] *= -1.0
        return b, nl

    def boundary_load(self, q: np.ndarray) -> np.ndarray:
        """Boundary term of Eq. weakform, int_{dOmega} (q . n) phi_i ds, for a
        nodal flux vector field q [n, 5, 2] (q = nu(u) grad u for the
        compartments), P1 along each boundary edge and integrated exactly:
        (2 q_i + q_j) . n L / 6 for node i of edge (i, j)."""
        b, nl = self.boundary_edges()
        i, j = b[:, 0], b[:, 1]
        qi = np.einsum("ecd,ed->ec", q[i], nl)
        qj = np.einsum("ecd,ed->ec", q[j], nl)
        out = np.zeros((self.n, q.shape[1]))
        np.add.at(out, i, (2.0 * qi + qj) / 6.0)
        np.add.at(out, j, (2.0 * qj + qi) / 6.0)
        return out


def params_vec(p) -> dict:
    return dict(sigma=p.sigma, gE=p.gamma_E, gR=p.gamma_R, gD=p.gamma_D,
                A=p.A, alpha=p.alpha, mu=p.mu, bI=p.beta_I, bE=p.beta_E,
                nu=np.asarray(p.nu, dtype=np.float64))


def reaction(u: np.ndarray, p, g=None) -> np.ndarray:
    """Nodal reaction B(u)u (Eq. vec_component2, equivalently the reaction
    parts of Eqs. seird1-5).  u [n,5] -> [n,5]."""
    q = params_vec(p)
    s, e, i, r, d = u.T
    N = s + e + i + r + d
    gg = 1.0 if g is None else g
    a = 1.0 - q["A"] / N                      # Allee factor
    lam = gg * (q["bI"] * i + q["bE"] * e)    # force of infection
    out = np.empty_like(u)
    out[:, 0] = q["alpha"] * N - a * lam * s - q["mu"] * s
    out[:, 1] = a * lam * s - (q["sigma"] + q["gE"] + q["mu"]) * e
    out[:, 2] = q["sigma"] * e - (q["gR"] + q["gD"] + q["mu"]) * i
    out[:, 3] = q["gE"] * e + q["gR"] * i - q["mu"] * r
    out[:, 4] = q["gD"] * i
    return out


def reaction_jacobian(u: np.ndarray, p, g=None) -> np.ndarray:
    """d(B(u)u)/du per node: [n,5,5], row = equation, column = unknown.
    The Allee factor depends on N, and dN/du_c = 1 for every c (Eq. N)."""
    q = params_vec(p)
    s, e, i, r, d = u.T
    N = s + e + i + r + d
    gg = np.ones_like(s) if g is None else np.broadcast_to(g, s.shape)
    a = 1.0 - q["A"] / N
    da = q["A"] / N ** 2                       # d a / d u_c, same for all c
    lam = gg * (q["bI"] * i + q["bE"] * e)
    dlam = np.zeros((len(s), NC))
    dlam[:, 2] = gg * q["bI"]
    dlam[:, 1] = gg * q["bE"]
    # d(a lam s)/du_c
    dals = (da * lam * s)[:, None] + (a * s)[:, None] * dlam
    dals[:, 0] += a * lam
    J = np.zeros((len(s), NC, NC))
    J[:, 0, :] = q["alpha"] - dals
    J[:, 0, 0] -= q["mu"]
    J[:, 1, :] = dals
    J[:, 1, 1] -= q["sigma"] + q["gE"] + q["mu"]
    J[:, 2, 1] = q["sigma"]
    J[:, 2, 2] = -(q["gR"] + q["gD"] + q["mu"])
    J[:, 3, 1] = q["gE"]
    J[:, 3, 2] = q["gR"]
    J[:, 3, 3] = -q["mu"]
    J[:, 4, 2] = q["gD"]
    return J


def diffusion(u: np.ndarray, geo: Geometry, nu) -> np.ndarray:
    """Diffusion term of the weak form, (nu(u) grad u, grad phi_i) for every
    node i and compartment c:  nu_c sum_T mean_T(N) sum_j K^T_ij u_{c,j}."""
    nu = np.asarray(nu, dtype=np.float64)
    N = u.sum(1)
    Nbar = N[geo.tri].mean(1)                          # [nt]
    ul = u[geo.tri]                                    # [nt, 3, 5]
    Ku = np.einsum("tkl,tlc->tkc", geo.K, ul)          # [nt, 3, 5]
    contrib = Nbar[:, None, None] * Ku * nu[None, None, :]
    out = np.zeros_like(u)
    np.add.at(out, geo.tri.ravel(), contrib.reshape(-1, NC))
    return out


def residual(u, u_prev, dt, geo: Geometry, p, g=None, src=None, mass="lumped", neumann=None):
    """Backward-Euler residual of the weak form (Eqs. timediscrete, weakform):

    F_{c,i} = m_i (u_{c,i} - u^n_{c,i}) + dt * diffusion_{c,i}(u)
              - dt * m_i * R_c(u_i) - dt * m_i * src_{c,i}
              - dt * int_{dOmega} gN_c phi_i ds

    ``src`` is an optional nodal forcing (used only by manufactured
    solutions).  mass = "consistent" replaces the lumped mass of the time
    derivative term by the consistent one, sum_j M_ij (u_j - u^n_j) (the
    reaction keeps nodal quadrature).  ``neumann`` [n, 5, 2]: nodal values
    of the flux vector nu(u) grad u whose normal component is Eq.
    weakform's boundary term (only boundary nodes matter; None:
    homogeneous Neumann)."""
    m = geo.mass[:, None]
    if mass == "consistent":
        Mt = geo.consistent_mass() @ (u - u_prev)
    else:
        Mt = m * (u - u_prev)
    F = Mt + dt * diffusion(u, geo, p.nu) - dt * m * reaction(u, p, g)
    if src is not None:
        F -= dt * m * src
    if neumann is not None:
        F -= dt * geo.boundary_load(neumann)
    return F


def jacobian(u, dt, geo: Geometry, p, g=None, mass_coef: float = 1.0, mass="lumped"):
    """Exact Jacobian dF/du of ``residual`` as a scipy CSR matrix of size
    5n x 5n (unknown 5*node + c).

    Diffusion block for an element T and local nodes k, l:
      d/du_{c',l} [nu_c Nbar_T sum_m K_km u_{c,m}]
        = nu_c Nbar_T K_kl delta_{cc'} + nu_c (1/3) sum_m K_km u_{c,m}
    (dNbar_T/du_{c',l} = 1/3 for every c').  Reaction and mass terms sit on
    the node's own 5x5 block."""
    nu = np.asarray(p.nu, dtype=np.float64)
    n = geo.n
    tri = geo.tri
    N = u.sum(1)
    Nbar = N[tri].mean(1)
    ul = u[tri]                                        # [nt,3,5]
    Ku = np.einsum("tkl,tlc->tkc", geo.K, ul)          # [nt,3,5] sum_m K_km u_cm
    rows, cols, vals = [], [], []
    for k in range(3):
        for l in range(3):
            for c in range(NC):
                if nu[c] == 0.0:
                    continue
                # diagonal-in-c part
                rows.append(5 * tri[:, k] + c)
                cols.append(5 * tri[:, l] + c)
                vals.append(dt * nu[c] * Nbar * geo.K[:, k, l])
                # dN part, same for all c'
                for cp in range(NC):
                    rows.append(5 * tri[:, k] + c)
                    cols.append(5 * tri[:, l] + cp)
                    vals.append(dt * nu[c] * Ku[:, k, c] / 3.0)
    # node blocks: mass - dt * m * dR/du
    JR = reaction_jacobian(u, p, g)
    m = geo.mass
    node = np.arange(n)
    for c in range(NC):
        for cp in range(NC):
            v = -dt * m * JR[:, c, cp]
            if c == cp and mass != "consistent":
                v = v + mass_coef * m
            rows.append(5 * node + c)
            cols.append(5 * node + cp)
            vals.append(v)
    if mass == "consistent":
        M = geo.consistent_mass().tocoo()
        for c in range(NC):
            rows.append(5 * M.row + c)
            cols.append(5 * M.col + c)
            vals.append(mass_coef * M.data)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    J = sp.coo_matrix((vals, (rows, cols)), shape=(NC * n, NC * n)).tocsr()
    J.sum_duplicates()
    return J


def beta_time_factor(t, a, b, k, tc):
    """Time factor of the transmission rate (Eq. beta_ie): a - b / (1 +
    exp(k (tc - t))); the paper's is a = 0.101, b = 0.05, k = 1, tc = 130
    days (the post-holiday lockdown)."""
    return a - b / (1.0 + np.exp(k * (tc - t)))


def beta_regional(x, beta_c, beta_e, beta_w, x_e, x_w, k_e=5.0, k_w=10.0):
    """Regional transmission profile along the first coordinate (Eq.
    beta_x): central value, with logistic steps to the eastern value past
    x_e and to the western value before x_w."""
    return (beta_c + (beta_e - beta_c) / (1.0 + np.exp(-k_e * (x - x_e)))
            + (beta_w - beta_c) / (1.0 + np.exp(k_w * (x - x_w))))


def node_graph(geo: Geometry) -> sp.csr_matrix:
    """Node adjacency (nodes sharing a triangle), including the diagonal."""
    tri = geo.tri
    r = np.repeat(tri, 3, axis=1).ravel()
    c = np.tile(tri, (1, 3)).ravel()
    G = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(geo.n, geo.n)).tocsr()
    G.data[:] = 1.0
    return G


def total_population(u, geo: Geometry) -> float:
    """sum_i m_i sum_c u_{c,i}: the discrete total population, conserved
    when alpha = mu = 0 (Section 2.1: isolated domain)."""
    return float(geo.mass @ u.sum(1))
