"""GMRES and overlapping Schwarz preconditioners (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

* ``gmres`` -- restarted GMRES(m) with right preconditioning, x0 = 0,
  modified Gram-Schmidt Arnoldi and Givens rotations; convergence when the
  residual norm drops below max(rtol ||b||, atol), divergence when it exceeds
  dtol ||b||, outer cap max_it (Section 3.2 stopping rules).
* ``RAS`` -- restricted additive Schwarz, M^{-1} = sum_i R_i^T D_i A_i^{-1}
  R_i with A_i = R_i A R_i^T and Boolean D_i (Eq. RAS); subdomains are the
  owner sets of a node partition grown by ``overlap`` layers of node-graph
  neighbours; local problems solved exactly (sparse LU).
* ``TwoLevel`` -- multiplicative two-grid preconditioner built from the
  three-step recurrence (Eqs. presmoother, coarsecorrection, postsmoother):
  pre-smooth with RAS, coarse correction Q = Z A_c^{-1} Z^T with the Galerkin
  coarse matrix A_c = Z^T A Z (Section 3.1), post-smooth with RAS.  Z is the
  P1 interpolation from a nested coarse grid, applied to each compartment.
* ``TwoLevelKrylov`` -- the same recurrence with the coarse system solved by
  GMRES preconditioned with RAS on the coarse graph ("Two-grid RAS - V2",
  Section 3.2), the outer solver being the flexible GMRES above (it keeps
  the preconditioned vectors); with ``inner="amg"`` the inner preconditioner
  is the aggregation AMG V-cycle of ``oracle/amg.py`` ("Two-grid RAS - V3").
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

NC = 5


def gmres(matvec, b, prec=None, restart=30, rtol=1e-5, atol=1e-50, dtol=1e5,
          max_it=200):
    """Returns (x, info) with info = dict(its, reason, resid)."""
    prec = (lambda v: v) if prec is None else prec
    n = len(b)
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    target = max(rtol * bnorm, atol)
    r = b.copy()
    beta = np.linalg.norm(r)
    its = 0
    if beta <= target:
        return x, dict(its=0, reason="converged", resid=beta)
    while True:
        m = restart
        V = np.zeros((m + 1, n))
        Zs = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        reason = None
        k = 0
        for j in range(m):
            Zs[j] = prec(V[j])
            w = matvec(Zs[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            if den == 0.0:
                reason = "breakdown"
                break
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            hnext = H[j + 1, j]
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            its += 1
            k = j + 1
            res = abs(gvec[j + 1])
            if res < target:
                reason = "converged"
                break
            if res > dtol * bnorm:
                reason = "diverged"
                break
            if its >= max_it:
                reason = "max_it"
                break
            if hnext == 0.0:
                reason = "converged"   # happy breakdown: exact solution
                break
            V[j + 1] = w / hnext
        if k > 0:
            y = np.linalg.solve(np.triu(H[:k, :k]), gvec[:k])
            x = x + Zs[:k].T @ y
        if reason is not None:
            r = b - matvec(x)
            return x, dict(its=its, reason=reason, resid=np.linalg.norm(r),
                           est=abs(gvec[k]))
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= target:
            return x, dict(its=its, reason="converged", resid=beta)


def grow_overlap(G: sp.csr_matrix, nodes: np.ndarray, layers: int) -> np.ndarray:
    """Node set grown by ``layers`` layers of graph neighbours."""
    mask = np.zeros(G.shape[0], dtype=bool)
    mask[nodes] = True
    for _ in range(layers):
        mask = (G @ mask.astype(np.float64)) > 0
    return np.nonzero(mask)[0]


def unknowns_of(nodes: np.ndarray, bs: int = NC) -> np.ndarray:
    return (bs * nodes[:, None] + np.arange(bs)[None, :]).ravel()


class RAS:
    """One-level restricted additive Schwarz with exact local solves.  bs:
    unknowns per node (5 for the coupled system, 1 for one compartment)."""

    def __init__(self, A: sp.csr_matrix, G: sp.csr_matrix, part: np.ndarray,
                 n_sub: int, overlap: int, bs: int = NC):
        self.A = A.tocsr()
        self.subs = []
        for i in range(n_sub):
            owned = np.nonzero(part == i)[0]
            if len(owned) == 0:
                continue
            nodes = grow_overlap(G, owned, overlap)
            idx = unknowns_of(nodes, bs)
            own = np.repeat(part[nodes] == i, bs)
            Ai = self.A[idx][:, idx].tocsc()
            lu = spla.splu(Ai)
            self.subs.append((idx, own, lu))

    def apply(self, r):
        z = np.zeros_like(r)
        for idx, own, lu in self.subs:
            zi = lu.solve(r[idx])
            z[idx[own]] = zi[own]
        return z

    def apply_T(self, r):
        """Transpose: sum_i R_i^T A_i^{-T} D_i R_i."""
        z = np.zeros_like(r)
        for idx, own, lu in self.subs:
            ri = np.where(own, r[idx], 0.0)
            z[idx] += lu.solve(ri, trans="T")
        return z


def nested_interpolation(parents_list, n_coarse: int) -> sp.csr_matrix:
    """Node-level P1 interpolation Z (n_fine x n_coarse) of a nested grid from
    its refinement records: a midpoint node takes the mean of its edge's two
    end values, an old node its own value.  Z is the product of the
    per-level interpolations."""
    Z = sp.identity(n_coarse, format="csr")
    for par in parents_list:
        n_l = len(par)
        n_prev = Z.shape[0]
        rows = np.repeat(np.arange(n_l), 2)
        cols = par.reshape(-1).astype(np.int64)
        vals = np.full(2 * n_l, 0.5)
        P = sp.coo_matrix((vals, (rows, cols)), shape=(n_l, n_prev)).tocsr()
        P.sum_duplicates()
        Z = P @ Z
    return Z.tocsr()


class TwoLevel:
    """Multiplicative two-grid RAS (pre-smooth, coarse correction,
    post-smooth)."""

    def __init__(self, A, ras: RAS, Znodes: sp.csr_matrix):
        self.A = A.tocsr()
        self.ras = ras
        self.Z = sp.kron(Znodes, sp.identity(NC), format="csr")
        self.Ac = (self.Z.T @ self.A @ self.Z).tocsc()
        self.lu = spla.splu(self.Ac)

    def coarse(self, r):
        return self.Z @ self.lu.solve(self.Z.T @ r)

    def coarse_T(self, r):
        return self.Z @ self.lu.solve(self.Z.T @ r, trans="T")

    def apply(self, r):
        z1 = self.ras.apply(r)
        r1 = r - self.A @ z1
        z2 = z1 + self.coarse(r1)
        r2 = r - self.A @ z2
        return z2 + self.ras.apply(r2)

    def apply_T(self, r):
        """Transpose of the operator above: the same three stages in the
        same order with A^T, M_RAS^T and Q^T (the error propagator
        (I - M A)(I - Q A)(I - M A) transposes to itself with the factors
        transposed)."""
        AT = self.A.T.tocsr()
        z1 = self.ras.apply_T(r)
        r1 = r - AT @ z1
        z2 = z1 + self.coarse_T(r1)
        r2 = r - AT @ z2
        return z2 + self.ras.apply_T(r2)


def make_linsolve(geo, part, n_sub, overlap, coarse=None, restart=30,
                  rtol=1e-5, atol=1e-50, dtol=1e5, max_it=200, G=None):
    """Newton linear solver J delta = -F by GMRES + (two-level) RAS, built
    afresh for every Jacobian.  ``coarse`` = (parents_list, n_coarse) or
    None.  Returns a callable (J, b) -> (x, info)."""
    from . import fem
    G = fem.node_graph(geo) if G is None else G
    Zn = None
    if coarse is not None:
        Zn = nested_interpolation(coarse[0], coarse[1])

    def solve(J, b):
        ras = RAS(J, G, part, n_sub, overlap)
        pc = ras if Zn is None else TwoLevel(J, ras, Zn)
        x, info = gmres(lambda v: J @ v, b, pc.apply, restart=restart,
                        rtol=rtol, atol=atol, dtol=dtol, max_it=max_it)
        return x, info

    return solve


def coarse_graph(Znodes: sp.csr_matrix, G: sp.csr_matrix) -> sp.csr_matrix:
    """Node graph of the Galerkin coarse matrix, including the diagonal (as
    ``fem.node_graph``): coarse nodes I and J are coupled when some fine a
    with Z_aI != 0 and b in {a} U adj(a) with Z_bJ != 0 exist, i.e. the
    pattern of Z^T (G + I) Z."""
    n = G.shape[0]
    Gi = (G + sp.identity(n, format="csr")).tocsr()
    Gi.data[:] = 1.0
    Zp = Znodes.copy().tocsr()
    Zp.data[:] = 1.0
    C = (Zp.T @ Gi @ Zp).tocsr()
    C.data[:] = 1.0
    return C


def coarse_partition(Znodes: sp.csr_matrix, part: np.ndarray, n_sub: int,
                     n_groups: int = 0) -> np.ndarray:
    """Coarse subdomain of every coarse node: the subdomain of the fine node
    with the largest interpolation weight in its column of Z (on a nested
    grid, the coarse node's own fine node; the lowest such fine index on a
    tie); with n_groups > 0 the fine subdomains s are merged into groups
    s * n_groups // n_sub.  Group numbers are then renumbered over the
    non-empty groups in increasing order."""
    Zc = Znodes.tocsc()
    owner = np.empty(Zc.shape[1], dtype=np.int64)
    for I in range(Zc.shape[1]):
        rows = Zc.indices[Zc.indptr[I]:Zc.indptr[I + 1]]
        vals = Zc.data[Zc.indptr[I]:Zc.indptr[I + 1]]
        order = np.lexsort((rows, -vals))  # largest weight, then lowest index
        owner[I] = part[rows[order[0]]]
    if n_groups > 0:
        owner = owner * n_groups // n_sub
    used = np.unique(owner)
    return np.searchsorted(used, owner), len(used)


class TwoLevelKrylov(TwoLevel):
    """Two-grid RAS with the coarse system A_c x = Z^T r solved by GMRES
    (x0 = 0, right preconditioning, restart, rtol/atol, max_it) with
    one-level RAS on the coarse graph (inner="ras"; the coarse subdomains are
    those of ``coarse_partition`` grown by ``overlap`` coarse-graph layers)
    or the aggregation AMG V-cycle (inner="amg"; ``amg`` holds its
    options).  ``infos`` collects the inner solves' reports."""

    def __init__(self, A, ras: RAS, Znodes: sp.csr_matrix, G: sp.csr_matrix,
                 part: np.ndarray, n_sub: int, n_groups: int = 0, overlap: int = 1,
                 restart: int = 30, max_it: int = 100, rtol: float = 1e-5,
                 atol: float = 1e-50, inner: str = "ras", amg=None):
        self.A = A.tocsr()
        self.ras = ras
        self.Z = sp.kron(Znodes, sp.identity(NC), format="csr")
        self.Ac = (self.Z.T @ self.A @ self.Z).tocsr()
        if inner == "amg":
            from .amg import AggregationAMG
            self.amg = AggregationAMG(self.Ac, coarse_graph(Znodes, G), **(amg or {}))
            self.ras_c = self.amg
            self.n_coarse_sub = 0
        else:
            cpart, nsc = coarse_partition(Znodes, part, n_sub, n_groups)
            self.ras_c = RAS(self.Ac, coarse_graph(Znodes, G), cpart, nsc, overlap)
            self.n_coarse_sub = nsc
        self.kw = dict(restart=restart, max_it=max_it, rtol=rtol, atol=atol, dtol=np.inf)
        self.infos = []

    def coarse(self, r):
        rc = self.Z.T @ r
        xc, info = gmres(lambda v: self.Ac @ v, rc, self.ras_c.apply, **self.kw)
        self.infos.append(info)
        return self.Z @ xc

    def coarse_T(self, r):
        raise NotImplementedError("the Krylov coarse solve has no transposed form")
