"""Algebraic multigrid V-cycle for the coarse problem of "Two-grid RAS - V3"
(oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Section 3.2 solves the coarse system of V3 with GMRES preconditioned by an
AMG V-cycle with a Jacobi smoother and Gaussian elimination on the last
level (BoomerAMG).  Readings where the paper only names the package:

* coarsening by plain aggregation of the node graph (all NC unknowns of a
  node go to the same aggregate), not classical Ruge-Stueben splitting:
  greedy in node order -- (1) a node none of whose neighbours is taken
  starts an aggregate with all of them; (2) every node still free joins
  the aggregate of its lowest-numbered taken neighbour (taken in (1));
  (3) a node left over (no taken neighbour) starts an aggregate of its own
  together with its free neighbours; aggregates are numbered in the order
  they start;
* prolongation piecewise constant on the aggregates, each unknown of a node
  taking its aggregate's value of the same component; restriction its
  transpose; Galerkin coarse matrices R A P;
* levels until a level has at most ``max_coarse`` nodes (or stops
  shrinking); the last level is solved exactly (dense LU);
* smoothing by damped Jacobi over the node blocks (the NC x NC diagonal
  block of a node inverted), ``nu`` sweeps before and after the coarse
  correction, damping ``omega``, starting from x = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla

NC = 5


def aggregate(G: sp.csr_matrix):
    """Aggregates of a node graph (diagonal ignored).  Returns agg[node]."""
    G = G.tocsr()
    n = G.shape[0]
    nbrs = [sorted(set(G.indices[G.indptr[i]:G.indptr[i + 1]].tolist()) - {i}) for i in range(n)]
    agg = -np.ones(n, dtype=np.int64)
    na = 0
    for i in range(n):                                     # (1)
        if agg[i] < 0 and all(agg[j] < 0 for j in nbrs[i]):
            agg[i] = na
            for j in nbrs[i]:
                agg[j] = na
            na += 1
    first = agg.copy()
    for i in range(n):                                     # (2)
        if agg[i] < 0:
            for j in nbrs[i]:
                if first[j] >= 0:
                    agg[i] = first[j]
                    break
    for i in range(n):                                     # (3)
        if agg[i] < 0:
            agg[i] = na
            for j in nbrs[i]:
                if agg[j] < 0:
                    agg[j] = na
            na += 1
    return agg


def tentative_prolongation(agg: np.ndarray, bs: int = NC) -> sp.csr_matrix:
    n = len(agg)
    na = int(agg.max()) + 1
    rows = np.arange(bs * n)
    cols = bs * np.repeat(agg, bs) + np.tile(np.arange(bs), n)
    return sp.csr_matrix((np.ones(bs * n), (rows, cols)), shape=(bs * n, bs * na))


def block_diag_inverse(A: sp.csr_matrix, bs: int = NC) -> sp.csr_matrix:
    n = A.shape[0] // bs
    blocks = []
    for i in range(n):
        idx = slice(bs * i, bs * i + bs)
        blocks.append(np.linalg.inv(A[idx, idx].toarray()))
    return sp.block_diag(blocks, format="csr")


class AggregationAMG:
    """V-cycle preconditioner z = V(r) for a node-block matrix A (bs unknowns
    per node) on the node graph G."""

    def __init__(self, A: sp.csr_matrix, G: sp.csr_matrix, max_coarse: int = 40, nu: int = 1,
                 omega: float = 2.0 / 3.0, bs: int = NC):
        self.bs, self.nu, self.omega = bs, nu, omega
        self.A = [A.tocsr()]
        self.P = []
        self.Dinv = []
        self.aggs = []
        Gl = G.tocsr()
        while Gl.shape[0] > max_coarse:
            agg = aggregate(Gl)
            na = int(agg.max()) + 1
            if na >= Gl.shape[0]:
                break
            P = tentative_prolongation(agg, bs)
            self.aggs.append(agg)
            self.P.append(P)
            self.Dinv.append(block_diag_inverse(self.A[-1], bs))
            self.A.append((P.T @ self.A[-1] @ P).tocsr())
            Pn = tentative_prolongation(agg, 1)
            Gl = (Pn.T @ (Gl + sp.identity(Gl.shape[0], format="csr")) @ Pn).tocsr()
            Gl.data[:] = 1.0
        self.lu = sla.lu_factor(self.A[-1].toarray())

    @property
    def levels(self):
        return len(self.A)

    def vcycle(self, b, level=0):
        if level == len(self.A) - 1:
            return sla.lu_solve(self.lu, b)
        A, Dinv, P = self.A[level], self.Dinv[level], self.P[level]
        x = np.zeros_like(b)
        for _ in range(self.nu):
            x = x + self.omega * (Dinv @ (b - A @ x))
        x = x + P @ self.vcycle(P.T @ (b - A @ x), level + 1)
        for _ in range(self.nu):
            x = x + self.omega * (Dinv @ (b - A @ x))
        return x

    def apply(self, r):
        return self.vcycle(r)
