"""Pins of the oracle's aggregation AMG (the coarse solver of "Two-grid RAS -
V3", Section 3.2): the aggregates, the Galerkin coarse matrix, the V-cycle
against its closed-form error propagator, exactness on one level, and the
V3 two-grid operator against the direct one."""
import numpy as np
import pytest
import scipy.sparse as sp

import seird_inputs as si
from oracle import amg, fem, krylov


@pytest.fixture(scope="module")
def coarse():
    cfg = si.config_nested_square(n_base=6, n_ref=2, n_sub=16)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    # dt = 1: block Jacobi converges on this coarse matrix (at dt = 10 the
    # reaction coupling gives D^{-1} A eigenvalues of negative real part)
    J = fem.jacobian(cfg.u0, 1.0, geo, cfg.params)
    G = fem.node_graph(geo)
    Zn = krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n)
    Z = sp.kron(Zn, sp.identity(5), format="csr")
    Ac = (Z.T @ J @ Z).tocsr()
    Gc = krylov.coarse_graph(Zn, G)
    return cfg, geo, J, G, Zn, Ac, Gc


def test_aggregates_partition_connected_node_sets(coarse):
    cfg, geo, J, G, Zn, Ac, Gc = coarse
    agg = amg.aggregate(Gc)
    n = Gc.shape[0]
    assert agg.min() == 0 and np.all(agg >= 0)
    assert set(agg.tolist()) == set(range(agg.max() + 1))
    assert agg.max() + 1 < n                       # it coarsens
    for a in range(agg.max() + 1):
        nodes = np.nonzero(agg == a)[0]
        # connected within the aggregate (breadth-first over G restricted)
        seen = {nodes[0]}
        front = [nodes[0]]
        S = set(nodes.tolist())
        while front:
            i = front.pop()
            for j in Gc.indices[Gc.indptr[i]:Gc.indptr[i + 1]]:
                if j in S and j not in seen:
                    seen.add(j)
                    front.append(j)
        assert seen == S, a


def test_galerkin_coarse_matrix_sums_the_aggregates_blocks(coarse):
    cfg, geo, J, G, Zn, Ac, Gc = coarse
    agg = amg.aggregate(Gc)
    P = amg.tentative_prolongation(agg)
    A1 = (P.T @ Ac @ P).toarray()
    na = agg.max() + 1
    B = np.zeros((5 * na, 5 * na))
    C = Ac.tocoo()
    for i, j, v in zip(C.row, C.col, C.data):       # brute force over the nonzeros
        B[5 * agg[i // 5] + i % 5, 5 * agg[j // 5] + j % 5] += v
    assert np.abs(A1 - B).max() <= 1e-12 * np.abs(B).max()


def test_one_level_is_an_exact_solve(coarse):
    cfg, geo, J, G, Zn, Ac, Gc = coarse
    M = amg.AggregationAMG(Ac, Gc, max_coarse=10 ** 6)
    assert M.levels == 1
    b = np.random.default_rng(1).standard_normal(Ac.shape[0])
    x = M.apply(b)
    assert np.linalg.norm(Ac @ x - b) <= 1e-12 * np.linalg.norm(b)


def _dense(apply, n):
    return np.column_stack([apply(e) for e in np.eye(n)])


def test_two_level_cycle_has_the_closed_form_error_propagator(coarse):
    """With two levels, I - B A = S^nu (I - P A_1^{-1} P^T A) S^nu with the
    smoother's propagator S = I - omega D^{-1} A (D the node blocks)."""
    cfg, geo, J, G, Zn, Ac, Gc = coarse
    for nu, omega in ((1, 2 / 3), (2, 0.5)):
        M = amg.AggregationAMG(Ac, Gc, max_coarse=Gc.shape[0] - 1, nu=nu, omega=omega)
        assert M.levels == 2
        n = Ac.shape[0]
        A = Ac.toarray()
        B = _dense(M.apply, n)
        D = np.zeros_like(A)
        for i in range(n // 5):
            D[5 * i:5 * i + 5, 5 * i:5 * i + 5] = A[5 * i:5 * i + 5, 5 * i:5 * i + 5]
        S = np.eye(n) - omega * np.linalg.solve(D, A)
        P = M.P[0].toarray()
        Q = np.eye(n) - P @ np.linalg.solve(P.T @ A @ P, P.T @ A)
        Sn = np.linalg.matrix_power(S, nu)
        E = Sn @ Q @ Sn
        assert np.abs((np.eye(n) - B @ A) - E).max() <= 1e-10
        # a dropped post-smoothing or a wrong damping would not satisfy it
        E_bad = Q @ Sn
        assert np.abs(E - E_bad).max() > 1e-3


def test_multilevel_cycle_is_a_convergent_iteration(coarse):
    cfg, geo, J, G, Zn, Ac, Gc = coarse
    M = amg.AggregationAMG(Ac, Gc, max_coarse=8)
    assert M.levels >= 3
    rng = np.random.default_rng(2)
    xs = rng.standard_normal(Ac.shape[0])
    b = Ac @ xs
    x = np.zeros_like(b)
    errs = []
    for _ in range(12):
        x = x + M.apply(b - Ac @ x)
        errs.append(np.linalg.norm(x - xs))
    assert errs[-1] < 1e-3 * errs[0]


def test_v3_with_an_exact_inner_solve_is_the_two_grid_operator(coarse):
    cfg, geo, J, G, Zn, Ac, Gc = coarse
    ras = krylov.RAS(J, G, cfg.part, cfg.n_sub, cfg.overlap)
    tl = krylov.TwoLevel(J, ras, Zn)
    tk = krylov.TwoLevelKrylov(J, ras, Zn, G, cfg.part, cfg.n_sub, inner="amg",
                               rtol=1e-15, atol=0.0, max_it=1000)
    r = np.random.default_rng(3).standard_normal(J.shape[0])
    a, b = tk.apply(r), tl.apply(r)
    assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)
    assert all(i["reason"] == "converged" for i in tk.infos)
    assert max(i["its"] for i in tk.infos) < 60
