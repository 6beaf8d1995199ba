"""Seeded synthetic inputs for the SEIRD implicit-step library and its oracle.

This module is shared by the oracle and the HIP path.  It holds only input
construction: meshes, refinement records, partitions, initial states,
parameter sets and configuration records.  It holds none of the method's
arithmetic (no element matrices, no residuals, no solvers).

Stand-ins for the paper's workloads (the paper's Southern Ontario geometry and
case data are not available):

* ``config_small``  -- unit square, structured right-triangle mesh, Gaussian
  infected bump, square-domain rates of the parameter table (Table 1),
  normalised so that the total density is 1 (Section 4.1 setup).
* ``config_realistic`` -- seeded star-shaped polygon of roughly 600 x 400 km,
  Delaunay base mesh refined by nested red refinement (the nested coarse grid
  of Section 3.1), log-normal density plus Gaussian urban peaks (the
  Gaussian-pulse initial densities of Section 4.3), Ontario-column rates of
  Table 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

S, E, I, R, D = range(5)
NCOMP = 5


# --------------------------------------------------------------------------
# parameter records
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    """Rate and diffusion parameters of the SEIRD system (Eqs. seird1-5).

    ``nu`` holds the five scalar diffusion coefficients nu_bar_c; the paper's
    deceased compartment does not diffuse, so ``nu[4]`` is 0 unless a caller
    sets it.  ``alpha`` and ``mu`` are the vital-dynamics rates (0 in the
    paper's studies)."""

    sigma: float
    gamma_E: float
    gamma_R: float
    gamma_D: float
    A: float
    beta_I: float
    beta_E: float
    nu: tuple
    alpha: float = 0.0
    mu: float = 0.0

    def as_array(self) -> np.ndarray:
        """Flat float64 layout shared with the C ABI ``seird_params``:
        sigma, gamma_E, gamma_R, gamma_D, A, alpha, mu, beta_I, beta_E, nu[5]."""
        return np.array([self.sigma, self.gamma_E, self.gamma_R, self.gamma_D,
                         self.A, self.alpha, self.mu, self.beta_I, self.beta_E,
                         *self.nu], dtype=np.float64)


def params_square() -> Params:
    """Square-domain column of Table 1, normalised to total density 1.

    The paper's values are in people/km^2 units with N = 2000; dividing
    densities by 2000 gives beta = 3.78e-4 * 2000 = 0.756 and A = 500 / 2000
    = 0.25.  Diffusion 1e-3 (S, E, I, R) as the small configuration states."""
    return Params(sigma=1 / 7, gamma_E=1 / 6, gamma_R=1 / 24, gamma_D=1 / 160,
                  A=0.25, beta_I=0.756, beta_E=0.756,
                  nu=(1e-3, 1e-3, 1e-3, 1e-3, 0.0))


def params_ontario() -> Params:
    """Ontario column of Table 1 (sigma 1/5, gamma_E 1/15, gamma_R 1/11,
    gamma_D 1/750) with transmission 0.01 and diffusion 0.05 km^2/day per
    density unit for S, E, R; the infected coefficient keeps the table's
    I:S ratio (1e-9 / 4.5e-7); the deceased do not diffuse."""
    nu_i = 0.05 * (1e-9 / 4.5e-7)
    return Params(sigma=1 / 5, gamma_E=1 / 15, gamma_R=1 / 11, gamma_D=1 / 750,
                  A=1e-3, beta_I=0.01, beta_E=0.01,
                  nu=(0.05, 0.05, nu_i, 0.05, 0.0))


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def square_mesh(nx: int, ny: Optional[int] = None, lx: float = 1.0,
                ly: float = 1.0):
    """Structured mesh of [0,lx]x[0,ly]: nx*ny cells, each split along the
    (i,j)->(i+1,j+1) diagonal into two counter-clockwise triangles.

    Nodes are numbered lexicographically, node (i, j) -> j*(nx+1) + i."""
    ny = nx if ny is None else ny
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys)  # [ny+1, nx+1]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v00 = (j * (nx + 1) + i).ravel()
    v10 = v00 + 1
    v01 = v00 + (nx + 1)
    v11 = v01 + 1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tri = np.empty((2 * nx * ny, 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    return xy, tri


def square_block_partition(nx: int, ny: int, bx: int, by: int) -> np.ndarray:
    """Owner subdomain of every node of ``square_mesh(nx, ny)`` for a bx x by
    block decomposition of the cells (nodes on the last line go to the last
    block)."""
    ii = np.arange(nx + 1)
    jj = np.arange(ny + 1)
    cx = np.minimum(ii * bx // nx, bx - 1)
    cy = np.minimum(jj * by // ny, by - 1)
    part = (cy[:, None] * bx + cx[None, :]).ravel()
    return part.astype(np.int32)


def star_polygon(seed: int, n_vert: int = 32, a: float = 300.0,
                 b: float = 200.0) -> np.ndarray:
    """Seeded star-shaped polygon: vertex k at angle theta_k (jittered) and
    radius ellipse(a, b; theta_k) * U(0.85, 1)."""
    rng = np.random.default_rng(seed)
    base = np.arange(n_vert) * (2 * np.pi / n_vert)
    theta = base + rng.uniform(-0.3, 0.3, n_vert) * (2 * np.pi / n_vert)
    theta = np.sort(theta)
    r_ell = a * b / np.sqrt((b * np.cos(theta)) ** 2 + (a * np.sin(theta)) ** 2)
    r = r_ell * rng.uniform(0.85, 1.0, n_vert)
    return np.stack([r * np.cos(theta), r * np.sin(theta)], axis=1)


def _points_in_polygon(p: np.ndarray, poly: np.ndarray) -> np.ndarray:
    """Even-odd ray casting test, vectorised over points."""
    x, y = p[:, 0], p[:, 1]
    inside = np.zeros(len(p), dtype=bool)
    n = len(poly)
    for k in range(n):
        x1, y1 = poly[k]
        x2, y2 = poly[(k + 1) % n]
        cond = (y1 > y) != (y2 > y)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = (x2 - x1) * (y - y1) / (y2 - y1) + x1
        inside ^= cond & (x < xint)
    return inside


def polygon_area(poly: np.ndarray) -> float:
    x, y = poly[:, 0], poly[:, 1]
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def delaunay_polygon_mesh(poly: np.ndarray, n_target: int, seed: int):
    """Delaunay mesh of a polygon: boundary points at spacing ~H plus a
    jittered grid of interior points (spacing H chosen so that roughly
    ``n_target`` nodes result); triangles whose centroid falls outside the
    polygon are dropped, unreferenced nodes removed, orientation made
    counter-clockwise."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    area = polygon_area(poly)
    H = math.sqrt(area / n_target)
    # boundary points
    bpts = []
    n = len(poly)
    for k in range(n):
        p0, p1 = poly[k], poly[(k + 1) % n]
        L = np.linalg.norm(p1 - p0)
        m = max(1, int(round(L / H)))
        t = np.arange(m) / m
        bpts.append(p0[None, :] + t[:, None] * (p1 - p0)[None, :])
    bpts = np.concatenate(bpts)
    lo = poly.min(0)
    hi = poly.max(0)
    gx = np.arange(lo[0] + H / 2, hi[0], H)
    gy = np.arange(lo[1] + H / 2, hi[1], H)
    GX, GY = np.meshgrid(gx, gy)
    g = np.stack([GX.ravel(), GY.ravel()], 1)
    g = g + rng.uniform(-0.3, 0.3, g.shape) * H
    g = g[_points_in_polygon(g, poly)]
    # keep interior points away from the boundary points
    from scipy.spatial import cKDTree

    dist, _ = cKDTree(bpts).query(g)
    g = g[dist > 0.5 * H]
    pts = np.concatenate([bpts, g])
    tri = Delaunay(pts).simplices
    cen = pts[tri].mean(1)
    tri = tri[_points_in_polygon(cen, poly)]
    # collinear boundary points give zero-area slivers: drop them (they
    # cover no area; a node left without triangles is removed below)
    p = pts[tri]
    det = np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                 - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    tri = tri[det > 1e-6 * H * H]
    used = np.unique(tri)
    remap = -np.ones(len(pts), dtype=np.int64)
    remap[used] = np.arange(len(used))
    pts = pts[used]
    tri = remap[tri]
    tri = _orient_ccw(pts, tri)
    return pts.astype(np.float64), tri.astype(np.int32)


def _orient_ccw(xy, tri):
    p = xy[tri]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - \
          (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    tri = tri.copy()
    neg = det < 0
    tri[neg, 1], tri[neg, 2] = tri[neg, 2].copy(), tri[neg, 1].copy()
    return tri


def red_refine(xy: np.ndarray, tri: np.ndarray):
    """One red refinement: every triangle is split into four by its edge
    midpoints.  Old nodes keep their numbers; new (midpoint) nodes follow.

    Returns (xy_fine, tri_fine, parents) where ``parents[a] = (p, q)`` names
    the two coarse nodes whose edge node ``a`` bisects, and (p, p) for an old
    node.  This is the refinement record from which a nested P1 coarse space
    is built; it carries no interpolation weights."""
    n = len(xy)
    nt = len(tri)
    a, b, c = tri[:, 0].astype(np.int64), tri[:, 1].astype(np.int64), tri[:, 2].astype(np.int64)
    edges = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1),
                            np.stack([c, a], 1)])
    es = np.sort(edges, axis=1)
    key = es[:, 0] * n + es[:, 1]
    ukey, inv = np.unique(key, return_inverse=True)
    mid = n + inv  # node index of the midpoint of each (triangle, edge)
    m_ab = mid[:nt]
    m_bc = mid[nt:2 * nt]
    m_ca = mid[2 * nt:]
    up = np.stack([ukey // n, ukey % n], 1)
    xy_new = 0.5 * (xy[up[:, 0]] + xy[up[:, 1]])
    xy_f = np.concatenate([xy, xy_new])
    tri_f = np.concatenate([
        np.stack([a, m_ab, m_ca], 1),
        np.stack([m_ab, b, m_bc], 1),
        np.stack([m_ca, m_bc, c], 1),
        np.stack([m_ab, m_bc, m_ca], 1),
    ]).astype(np.int32)
    parents = np.concatenate([np.stack([np.arange(n), np.arange(n)], 1), up])
    return xy_f, tri_f, parents.astype(np.int32)


def rcb_order(xy: np.ndarray, n_parts: int, leaf: int = 64):
    """Recursive coordinate bisection.

    Returns (order, part): ``order`` is a permutation of the nodes (a
    locality-preserving numbering, parts contiguous), ``part[k]`` is the
    owner part of node ``k`` in the ORIGINAL numbering.  Splits are along the
    longer extent of the bounding box at the (proportional) median; ties are
    broken by node index (stable sort)."""
    n = len(xy)
    part = np.zeros(n, dtype=np.int32)
    out = []

    def rec(idx, p0, np_):
        if np_ == 1:
            part[idx] = p0
            # finer ordering inside the part for locality
            out.append(_rcb_leaf_order(xy, idx, leaf))
            return
        pts = xy[idx]
        ext = pts.max(0) - pts.min(0)
        ax = 0 if ext[0] >= ext[1] else 1
        o = np.argsort(pts[:, ax], kind="stable")
        nl = np_ // 2
        cut = int(round(len(idx) * nl / np_))
        rec(idx[o[:cut]], p0, nl)
        rec(idx[o[cut:]], p0 + nl, np_ - nl)

    rec(np.arange(n), 0, n_parts)
    return np.concatenate(out), part


def _rcb_leaf_order(xy, idx, leaf):
    if len(idx) <= leaf:
        return idx
    stack = [idx]
    res = []
    while stack:
        cur = stack.pop()
        if len(cur) <= leaf:
            res.append(cur)
            continue
        pts = xy[cur]
        ext = pts.max(0) - pts.min(0)
        ax = 0 if ext[0] >= ext[1] else 1
        o = np.argsort(pts[:, ax], kind="stable")
        h = len(cur) // 2
        # push right first so that left is processed first
        stack.append(cur[o[h:]])
        stack.append(cur[o[:h]])
    return np.concatenate(res)


# ---------------------------------------------------------------------------
# 22-compartment model (Appendix C): compartments, synthetic rates, state
# ---------------------------------------------------------------------------
COMPARTMENTS22 = ["S", "V", "E", "Q", "A", "W", "F", "B", "C", "X", "Y", "Z", "G", "N", "H", "H1", "I",
                  "H2", "R1", "R2", "P", "D"]
DIFFUSING22 = ["S", "V", "E", "A", "F", "B", "C", "P", "R1", "R2"]


@dataclasses.dataclass
class Params22:
    """Parameters of the 22-compartment model (names of its parameter
    table; phi_C as in its equations).  The paper gives no values: these are
    synthetic rates per day of a plausible size.  beta_* weigh the four
    moving, non-isolating infectious compartments in the force of
    infection; ``nu`` holds the diffusion coefficients of S V E A F B C P R1
    R2 in that order."""
    beta_A: float = 0.3
    beta_F: float = 0.2
    beta_B: float = 0.3
    beta_C: float = 0.1
    r_V: float = 0.7
    delta_S: float = 0.1
    delta_V: float = 0.15
    gamma_A: float = 1 / 7
    gamma_C: float = 1 / 60
    gamma_DA: float = 0.05
    gamma_DM: float = 0.2
    gamma_E: float = 1 / 3
    gamma_I: float = 1 / 10
    gamma_L: float = 2e-4
    gamma_M: float = 1 / 7
    gamma_P: float = 1 / 2
    gamma_R: float = 1 / 180
    gamma_S1: float = 1 / 5
    gamma_S2: float = 1 / 10
    gamma_T: float = 1 / 200
    gamma_V: float = 5e-3
    sigma_A: float = 0.4
    sigma_C: float = 0.2
    sigma_H: float = 0.9
    sigma_S: float = 0.05
    pi_A: float = 1 / 3
    pi_B: float = 1 / 10
    pi_C: float = 1 / 7
    pi_H: float = 1 / 8
    phi_C: float = 0.1
    phi_M: float = 0.05
    phi_S: float = 0.2
    phi_P: float = 0.1
    kappa_H: float = 0.1
    kappa_I: float = 0.3
    kappa_N: float = 0.5
    kappa_P: float = 0.01
    nu: tuple = (1e-3, 1e-3, 1e-3, 5e-4, 5e-4, 2e-4, 1e-4, 2e-4, 1e-3, 1e-3)


def state22(xy: np.ndarray, seed: int = 0, peak: float = 1e-2, width: float = 0.1,
            jitter: float = 0.0) -> np.ndarray:
    """[n, 22] initial densities: total 1 per unit area, a seeded bump of
    exposed (60%) and presymptomatic (40%) people, 20% of the rest
    vaccinated, the others susceptible; ``jitter`` > 0 adds seeded
    nonnegative noise to every compartment (test states)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, 2)
    r2 = ((xy - c[None, :]) ** 2).sum(1)
    bump = peak * np.exp(-r2 / (2 * width ** 2))
    ix = {nm: k for k, nm in enumerate(COMPARTMENTS22)}
    u = np.zeros((len(xy), len(COMPARTMENTS22)))
    u[:, ix["E"]] = 0.6 * bump
    u[:, ix["A"]] = 0.4 * bump
    u[:, ix["V"]] = 0.2 * (1.0 - bump)
    if jitter > 0:
        u += jitter * rng.uniform(0.0, 1.0, u.shape)
    u[:, ix["S"]] = np.maximum(1.0 - (u.sum(1) - u[:, ix["S"]]), 0.0)
    return u


@dataclasses.dataclass
class NestedMesh:
    """A mesh obtained by ``n_ref`` red refinements of a base mesh.

    ``levels[l] = (xy, tri)`` for l = 0 (base) .. n_ref (finest);
    ``parents[l]`` (l >= 1) is the refinement record mapping level-l nodes
    to level-(l-1) node pairs.  The finest level may be renumbered; its
    ``parents`` rows follow that numbering."""

    levels: list
    parents: list

    @property
    def xy(self):
        return self.levels[-1][0]

    @property
    def tri(self):
        return self.levels[-1][1]

    def renumber_finest(self, order):
        """Renumber the finest level so that new node k is old node order[k]."""
        xy, tri = self.levels[-1]
        inv = np.empty(len(order), dtype=np.int64)
        inv[order] = np.arange(len(order))
        self.levels[-1] = (xy[order], inv[tri].astype(np.int32))
        if len(self.parents) > 0 and self.parents[-1] is not None:
            self.parents[-1] = self.parents[-1][order]


def nested_polygon_mesh(seed: int, n_base: int, n_ref: int,
                        a: float = 300.0, b: float = 200.0) -> NestedMesh:
    poly = star_polygon(seed, a=a, b=b)
    xy, tri = delaunay_polygon_mesh(poly, n_base, seed + 1000)
    levels = [(xy, tri)]
    parents = [None]
    for _ in range(n_ref):
        xy, tri, par = red_refine(xy, tri)
        levels.append((xy, tri))
        parents.append(par)
    return NestedMesh(levels=levels, parents=parents)


def nested_square_mesh(n_base: int, n_ref: int) -> NestedMesh:
    xy, tri = square_mesh(n_base)
    levels = [(xy, tri)]
    parents = [None]
    for _ in range(n_ref):
        xy, tri, par = red_refine(xy, tri)
        levels.append((xy, tri))
        parents.append(par)
    return NestedMesh(levels=levels, parents=parents)


# --------------------------------------------------------------------------
# initial states
# --------------------------------------------------------------------------
def gaussian_bump_state(xy: np.ndarray, seed: int, N0: float = 1.0,
                        peak: float = 1e-3, width: float = 0.05):
    """u0 [n,5]: uniform total density N0, infected Gaussian bump of the given
    peak and width at a seeded centre in [0.25, 0.75]^2, s = N0 - i,
    e = r = d = 0."""
    rng = np.random.default_rng(seed)
    xc = rng.uniform(0.25, 0.75, 2)
    r2 = ((xy - xc[None, :]) ** 2).sum(1)
    i0 = peak * N0 * np.exp(-r2 / (2 * width ** 2))
    u = np.zeros((len(xy), NCOMP))
    u[:, I] = i0
    u[:, S] = N0 - i0
    return u


def urban_density_state(xy: np.ndarray, poly_seed: int, noise_seed: int,
                        peak_seed: int, n_peaks: int = 12, n_seeded: int = 5,
                        clip: float = 3.0, a: float = 300.0, b: float = 200.0):
    """u0 [n,5] for the realistic configuration.

    Density N0 = exp(Z) + sum_k a_k exp(-|x-c_k|^2 / (2 rho_k^2)) with Z iid
    standard normal per node, clipped to [-clip, clip]; a_k ~ U(20, 100),
    rho_k ~ U(5, 25) km, c_k uniform in the polygon.  Infected density
    1e-3 * N0 * sum_{k < n_seeded} exp(-|x-c_k|^2/(2 rho_k^2)) (the
    Gaussian-pulse initial state of Section 4.3, with the exponent's minus
    sign), s = N0 - i."""
    poly = star_polygon(poly_seed, a=a, b=b)
    rng_z = np.random.default_rng(noise_seed)
    Z = np.clip(rng_z.standard_normal(len(xy)), -clip, clip)
    rng = np.random.default_rng(peak_seed)
    lo, hi = poly.min(0), poly.max(0)
    centres = []
    while len(centres) < n_peaks:
        c = rng.uniform(lo, hi, (64, 2))
        c = c[_points_in_polygon(c, poly)]
        centres.extend(list(c))
    centres = np.array(centres[:n_peaks])
    amp = rng.uniform(20.0, 100.0, n_peaks)
    rho = rng.uniform(5.0, 25.0, n_peaks)
    N0 = np.exp(Z)
    inf = np.zeros(len(xy))
    for k in range(n_peaks):
        g = np.exp(-((xy - centres[k]) ** 2).sum(1) / (2 * rho[k] ** 2))
        N0 += amp[k] * g
        if k < n_seeded:
            inf += g
    i0 = 1e-3 * N0 * inf
    u = np.zeros((len(xy), NCOMP))
    u[:, I] = i0
    u[:, S] = N0 - i0
    return u


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Config:
    name: str
    xy: np.ndarray
    tri: np.ndarray
    u0: np.ndarray
    params: Params
    dt: float
    steps: int
    part: np.ndarray          # owner subdomain per node
    n_sub: int
    overlap: int
    newton_tol: float = 1e-10
    newton_max_it: int = 20
    gmres_restart: int = 30
    gmres_rtol: float = 1e-5
    gmres_atol: float = 1e-50
    gmres_dtol: float = 1e5
    gmres_max_it: int = 200
    # nested coarse space: refinement records from the coarse level to the
    # finest level (list of [n_l, 2] int32 arrays), None for one level
    coarse_parents: Optional[List[np.ndarray]] = None
    coarse_n: int = 0

    @property
    def n(self):
        return len(self.xy)


def config_small(seed: int = 0, nx: int = 64) -> Config:
    """Plain FP64 small case: 64x64 structured unit-square mesh (4225 nodes),
    Gaussian infected bump (sigma 0.05, peak 1e-3) at a seeded centre,
    square-domain rates, dt 0.1, 10 steps, Newton tol 1e-10, GMRES(30) with
    one-level RAS on 4x4 = 16 blocks, overlap 1."""
    xy, tri = square_mesh(nx)
    u0 = gaussian_bump_state(xy, seed)
    part = square_block_partition(nx, nx, 4, 4)
    return Config(name=f"square{nx}", xy=xy, tri=tri, u0=u0,
                  params=params_square(), dt=0.1, steps=10, part=part,
                  n_sub=16, overlap=1)


def config_nested_square(n_base: int = 8, n_ref: int = 2, n_sub: int = 16,
                         seed: int = 0, overlap: int = 1,
                         coarse_level: int = 0) -> Config:
    """Small nested structured mesh with a two-level (nested coarse grid)
    preconditioner: base n_base x n_base square refined n_ref times, RCB
    partition into n_sub parts."""
    nm = nested_square_mesh(n_base, n_ref)
    order, part = rcb_order(nm.xy, n_sub)
    nm.renumber_finest(order)
    part = part[order]
    xy, tri = nm.xy, nm.tri
    u0 = gaussian_bump_state(xy, seed)
    return Config(name=f"nsquare{n_base}x{n_ref}", xy=xy, tri=tri, u0=u0,
                  params=params_square(), dt=0.1, steps=10, part=part,
                  n_sub=n_sub, overlap=overlap,
                  coarse_parents=nm.parents[coarse_level + 1:],
                  coarse_n=len(nm.levels[coarse_level][0]))


def config_realistic(n_base: int = 3900, n_ref: int = 4, n_sub: int = 1024,
                     overlap: int = 2, coarse_level: int = 0,
                     steps: int = 30, seed: int = 1) -> Config:
    """Realistic case: seeded star polygon (~600 x 400 km), Delaunay base mesh
    of ~n_base nodes red-refined n_ref times (about 1M nodes at the defaults),
    log-normal density with 12 urban peaks, infected at 5 peaks, Ontario
    rates, 30 daily steps, two-level RAS with RCB subdomains."""
    nm = nested_polygon_mesh(seed, n_base, n_ref)
    order, part = rcb_order(nm.xy, n_sub)
    nm.renumber_finest(order)
    part = part[order]
    xy, tri = nm.xy, nm.tri
    u0 = urban_density_state(xy, poly_seed=seed, noise_seed=seed + 1,
                             peak_seed=seed + 2)
    cp = nm.parents[coarse_level + 1:] if coarse_level is not None else None
    cn = len(nm.levels[coarse_level][0]) if coarse_level is not None else 0
    return Config(name=f"polygon{len(xy)}", xy=xy, tri=tri, u0=u0,
                  params=params_ontario(), dt=1.0, steps=steps, part=part,
                  n_sub=n_sub, overlap=overlap, coarse_parents=cp,
                  coarse_n=cn)


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


# --------------------------------------------------------------------------
# differentiation workload
# --------------------------------------------------------------------------
def voronoi_regions(xy: np.ndarray, n_regions: int, seed: int,
                    poly: Optional[np.ndarray] = None) -> np.ndarray:
    """Observation regions: Voronoi cells of ``n_regions`` seeded points
    (uniform in the mesh's bounding box, or in ``poly``); region id per
    node."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    lo, hi = xy.min(0), xy.max(0)
    pts = []
    while len(pts) < n_regions:
        c = rng.uniform(lo, hi, (4 * n_regions, 2))
        if poly is not None:
            c = c[_points_in_polygon(c, poly)]
        pts.extend(list(c))
    pts = np.array(pts[:n_regions])
    _, idx = cKDTree(pts).query(xy)
    return idx.astype(np.int32)


def bump_field(xy: np.ndarray, seed: int, n_bumps: int = 8,
               amp: float = 0.2, width: float = 40.0) -> np.ndarray:
    """Seeded smooth perturbation 1 + amp * tanh(sum of n_bumps Gaussian
    bumps with random signs): the 'truth' transmission multiplier."""
    rng = np.random.default_rng(seed)
    lo, hi = xy.min(0), xy.max(0)
    c = rng.uniform(lo, hi, (n_bumps, 2))
    sgn = rng.choice([-1.0, 1.0], n_bumps)
    w = rng.uniform(0.5, 1.5, n_bumps) * width
    xi = np.zeros(len(xy))
    for k in range(n_bumps):
        xi += sgn[k] * np.exp(-((xy - c[k]) ** 2).sum(1) / (2 * w[k] ** 2))
    return 1.0 + amp * np.tanh(xi)


def params22_realistic() -> "Params22":
    """Rates of ``Params22`` for the realistic polygon, whose densities reach
    ~130 per unit: transmission weights divided by 100 (so that beta times
    the largest densities stays below about 0.4 per day, as on the unit
    square with density 1) and constant diffusion coefficients in km^2/day
    (the five-compartment case's 0.05 per density unit times a typical
    density of 10)."""
    return Params22(beta_A=3e-3, beta_F=2e-3, beta_B=3e-3, beta_C=1e-3,
                    nu=(0.5, 0.5, 0.5, 0.25, 0.25, 0.1, 0.02, 0.1, 0.5, 0.5))


def state22_from(u5: np.ndarray) -> np.ndarray:
    """[n, 22] state from a five-compartment state [n, 5] (S E I R D): the
    total density is kept, the exposed stay exposed, the infected become
    presymptomatic, the recovered R1, the deceased D, and 20% of the
    susceptible are vaccinated."""
    ix = {nm: k for k, nm in enumerate(COMPARTMENTS22)}
    u = np.zeros((len(u5), len(COMPARTMENTS22)))
    u[:, ix["S"]] = 0.8 * u5[:, 0]
    u[:, ix["V"]] = 0.2 * u5[:, 0]
    u[:, ix["E"]] = u5[:, 1]
    u[:, ix["A"]] = u5[:, 2]
    u[:, ix["R1"]] = u5[:, 3]
    u[:, ix["D"]] = u5[:, 4]
    return u


@dataclasses.dataclass
class BatchConfig:
    """An ensemble of independent instances stepped together."""
    name: str
    instances: list           # Config records (one-level, no coarse space)
    dt: float
    steps: int
    overlap: int

    @property
    def n(self):
        return sum(c.n for c in self.instances)


def config_batch(n_inst: int = 48, n_min: float = 50_000, n_max: float = 400_000,
                 seed: int = 4, param_seed: int = 5, nodes_per_sub: int = 1000,
                 overlap: int = 2, n_ref: int = 2, steps: int = 30,
                 ref_nodes: float = 1.0e6, beta_base: float = 0.006) -> BatchConfig:
    """Ensemble case: ``n_inst`` realistic-type instances whose target node
    counts are log-uniform in [n_min, n_max] (``seed``).

    Instance k: star polygon seeded 100 + k with both semi-axes scaled by
    sqrt(n_k / ref_nodes), so that its node density matches the realistic
    case (about 1M nodes on the unscaled polygon); Delaunay base mesh of
    n_k / 4^n_ref nodes red-refined n_ref times; density and urban peaks as
    in the realistic case (seeds 100 + k, 101 + k, 102 + k), with the number
    of peaks (12, 5 of them seeded with infection, on the unscaled polygon)
    scaled by the area so that peaks per km^2 match it; Ontario rates
    with the transmission rates (beta_I = beta_E = beta_base times one
    U(0.7, 1.3) draw) and each diffusion coefficient nu_c scaled by its own
    U(0.7, 1.3) draw (``param_seed``).  beta_base is below the realistic
    case's 0.01 so that dt * beta * max N stays below 1 on every instance
    (as it does in the realistic case): beyond 1 + dt (sigma + gamma_E) the
    exposed equation's backward-Euler root turns negative.  RCB subdomains of about ``nodes_per_sub`` nodes,
    overlap 2; dt 1 day."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_inst))
    prng = np.random.default_rng(param_seed)
    fb = prng.uniform(0.7, 1.3, n_inst)
    fnu = prng.uniform(0.7, 1.3, (n_inst, NCOMP))
    base = params_ontario()
    out = []
    for k in range(n_inst):
        sc = math.sqrt(sizes[k] / ref_nodes)
        a, b = 300.0 * sc, 200.0 * sc
        nm = nested_polygon_mesh(100 + k, max(16, int(sizes[k] / 4 ** n_ref)), n_ref, a=a, b=b)
        n_sub = max(1, int(round(len(nm.xy) / nodes_per_sub)))
        order, part = rcb_order(nm.xy, n_sub)
        nm.renumber_finest(order)
        part = part[order]
        xy, tri = nm.xy, nm.tri
        n_peaks = max(1, int(round(12 * sc * sc)))
        u0 = urban_density_state(xy, poly_seed=100 + k, noise_seed=101 + k,
                                 peak_seed=102 + k, a=a, b=b, n_peaks=n_peaks,
                                 n_seeded=max(1, int(round(n_peaks * 5 / 12))))
        p = Params(**{**base.__dict__, "beta_I": beta_base * fb[k],
                      "beta_E": beta_base * fb[k],
                      "nu": tuple(np.array(base.nu) * fnu[k])})
        out.append(Config(name=f"inst{k}_{len(xy)}", xy=xy, tri=tri, u0=u0, params=p,
                          dt=1.0, steps=steps, part=part, n_sub=n_sub, overlap=overlap))
    tot = sum(c.n for c in out)
    return BatchConfig(name=f"ensemble{n_inst}x{tot}", instances=out, dt=1.0,
                       steps=steps, overlap=overlap)


def config_differentiation(n_base: int = 7800, n_ref: int = 4, n_sub: int = 2048,
                           steps: int = 60, seed: int = 6, beta: float = 0.006) -> Config:
    """Differentiation case: realistic-type mesh of about 2M nodes (10M
    unknowns), 60 daily steps, two-grid RAS; regions and truth field are
    built by ``voronoi_regions`` (40 regions, seed 8) and ``bump_field``
    (seed 7).  The base transmission is ``beta`` (0.006) instead of the
    realistic case's 0.01: this seed's densest node has N of about 151, and
    with the truth field's +20% the product dt * beta * g * N must stay
    below 1 (as in the realistic case) for the exposed equation's
    backward-Euler root to stay positive."""
    cfg = config_realistic(n_base=n_base, n_ref=n_ref, n_sub=n_sub, steps=steps, seed=seed)
    cfg.params = Params(**{**cfg.params.__dict__, "beta_I": beta, "beta_E": beta})
    return cfg
