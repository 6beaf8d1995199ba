"""Pins of the oracle's GMRES and Schwarz preconditioners (CPU only)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import seird_inputs as si
from oracle import fem, krylov, newton


def _system(cfg):
    geo = fem.Geometry(cfg.xy, cfg.tri)
    J = fem.jacobian(cfg.u0, cfg.dt, geo, cfg.params)
    b = np.random.default_rng(0).standard_normal(J.shape[0])
    return geo, J, b


def test_partition_of_unity():
    """sum_i R_i^T D_i R_i = I (Eq. RAS, Boolean D_i)."""
    cfg = si.config_small(nx=16)
    geo, J, _ = _system(cfg)
    ras = krylov.RAS(J, fem.node_graph(geo), cfg.part, cfg.n_sub, 2)
    acc = np.zeros(J.shape[0])
    for idx, own, _ in ras.subs:
        acc[idx[own]] += 1.0
    assert np.all(acc == 1.0)


def test_one_subdomain_is_exact_inverse():
    """One subdomain: RAS is A^{-1}, GMRES converges in one iteration."""
    cfg = si.config_small(nx=16)
    geo, J, b = _system(cfg)
    part = np.zeros(geo.n, dtype=np.int32)
    ras = krylov.RAS(J, fem.node_graph(geo), part, 1, 1)
    x, info = krylov.gmres(lambda v: J @ v, b, ras.apply, rtol=1e-12)
    assert info["its"] == 1
    assert np.linalg.norm(J @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_gmres_unpreconditioned_matches_direct():
    cfg = si.config_small(nx=16)
    geo, J, b = _system(cfg)
    x, info = krylov.gmres(lambda v: J @ v, b, None, restart=30, rtol=1e-12,
                           max_it=2000)
    assert info["reason"] == "converged"
    xd = spla.spsolve(J.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_gmres_minimises_residual_over_krylov_space():
    """Brute force on a tiny dense system: after k unrestarted steps the
    GMRES residual equals the least-squares minimum over span{b, Ab, ...}."""
    rng = np.random.default_rng(3)
    A = np.eye(12) * 3 + rng.standard_normal((12, 12))
    b = rng.standard_normal(12)
    for k in (2, 4, 6):
        x, info = krylov.gmres(lambda v: A @ v, b, None, restart=k, max_it=k,
                               rtol=1e-300)
        K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(k)], 1)
        c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
        best = np.linalg.norm(b - A @ K @ c)
        assert np.linalg.norm(b - A @ x) == __import__("pytest").approx(best, rel=1e-8)


def test_two_level_with_identity_coarse_space_is_exact():
    """Z = I makes the coarse correction exact: the multiplicative two-grid
    preconditioner is A^{-1} and GMRES needs one iteration."""
    cfg = si.config_small(nx=12)
    geo, J, b = _system(cfg)
    ras = krylov.RAS(J, fem.node_graph(geo), cfg.part, cfg.n_sub, 1)
    tl = krylov.TwoLevel(J, ras, sp.identity(geo.n, format="csr"))
    x, info = krylov.gmres(lambda v: J @ v, b, tl.apply, rtol=1e-11)
    assert info["its"] == 1


def test_nested_interpolation_reproduces_linear_functions():
    """P1 interpolation from a nested coarse grid is exact for linear
    functions (the coarse space contains them)."""
    nm = si.nested_square_mesh(4, 2)
    Z = krylov.nested_interpolation(nm.parents[1:], len(nm.levels[0][0]))
    xc = nm.levels[0][0]
    xf = nm.xy
    f = lambda p: 2.0 * p[:, 0] - 3.0 * p[:, 1] + 0.5
    assert np.allclose(Z @ f(xc), f(xf))
    assert np.allclose(Z.sum(1), 1.0)


def test_two_level_transpose_is_the_adjoint_operator():
    """<M^T x, y> = <x, M y> for the two-level preconditioner."""
    cfg = si.config_nested_square(n_base=4, n_ref=2, n_sub=4)
    geo, J, _ = _system(cfg)
    ras = krylov.RAS(J, fem.node_graph(geo), cfg.part, cfg.n_sub, cfg.overlap)
    Zn = krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n)
    tl = krylov.TwoLevel(J, ras, Zn)
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
    assert np.dot(tl.apply_T(x), y) == __import__("pytest").approx(np.dot(x, tl.apply(y)), rel=1e-10)
    assert np.dot(ras.apply_T(x), y) == __import__("pytest").approx(np.dot(x, ras.apply(y)), rel=1e-10)


def test_newton_gmres_ras_reaches_direct_root():
    cfg = si.config_small(nx=32)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    ls = krylov.make_linsolve(geo, cfg.part, cfg.n_sub, cfg.overlap)
    u1, info = newton.newton_step(cfg.u0, cfg.dt, geo, cfg.params, linsolve=ls)
    u2, _ = newton.newton_step(cfg.u0, cfg.dt, geo, cfg.params)
    assert np.abs(u1 - u2).max() <= 1e-9 * np.abs(u2).max()
    assert all(li["reason"] == "converged" for li in info["lin"])


# ---------------------------------------------------------------------------
# Pins of the restricted prolongation (Eq. RAS: Boolean D_i) and of the
# three-step two-grid operator (Eqs. presmoother, coarsecorrection,
# postsmoother), each with a planted mistake that the pin must catch.
# ---------------------------------------------------------------------------

def _decoupled_system(overlap):
    """Jacobian of the small square with every coupling between nodes of
    different owner subdomains removed: the matrix is block diagonal over
    the partition, while the subdomains still overlap in the mesh graph."""
    cfg = si.config_small(nx=16)
    geo, J, b = _system(cfg)
    node = np.arange(J.shape[0]) // krylov.NC
    Jc = J.tocoo()
    keep = cfg.part[node[Jc.row]] == cfg.part[node[Jc.col]]
    Jd = sp.coo_matrix((Jc.data[keep], (Jc.row[keep], Jc.col[keep])), shape=J.shape).tocsr()
    ras = krylov.RAS(Jd, fem.node_graph(geo), cfg.part, cfg.n_sub, overlap)
    return Jd, ras, b


def _asm_apply(ras, r):
    """Additive Schwarz without the restriction D_i: every local copy is
    added back (the mistake the owner-only prolongation must not make)."""
    z = np.zeros_like(r)
    for idx, own, lu in ras.subs:
        z[idx] += lu.solve(r[idx])
    return z


def _ras_error_on_decoupled(apply, overlap):
    Jd, ras, b = _decoupled_system(overlap)
    x = spla.spsolve(Jd.tocsc(), b)
    return np.linalg.norm(apply(ras, b) - x) / np.linalg.norm(x)


def test_ras_is_exact_on_a_matrix_decoupled_along_the_partition():
    """With A block diagonal over the owner sets, each local matrix splits
    into the owned block and an unrelated overlap block, so the owned part of
    A_i^{-1} R_i r is exactly (A^{-1} r) on the owned nodes: RAS (D_i = owner
    indicator) returns A^{-1} r.  Adding every copy (ASM) does not."""
    for overlap in (1, 2):
        assert _ras_error_on_decoupled(krylov.RAS.apply, overlap) <= 1e-12
        assert _ras_error_on_decoupled(_asm_apply, overlap) >= 1e-3


def test_planted_asm_prolongation_is_caught(monkeypatch):
    """Plant the ASM prolongation in the oracle's RAS: the decoupled-matrix
    pin fails, and so does the transposed operator's adjointness."""
    monkeypatch.setattr(krylov.RAS, "apply", lambda self, r: _asm_apply(self, r))
    assert _ras_error_on_decoupled(krylov.RAS.apply, 1) > 1e-3
    cfg = si.config_small(nx=16)
    geo, J, _ = _system(cfg)
    ras = krylov.RAS(J, fem.node_graph(geo), cfg.part, cfg.n_sub, 2)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
    lhs, rhs = np.dot(ras.apply_T(x), y), np.dot(x, ras.apply(y))
    assert abs(lhs - rhs) > 1e-6 * abs(rhs)


def _dense(op, n):
    return np.stack([op(e) for e in np.eye(n)], 1)


def _two_level_pieces():
    # dt = 10: diffusion strong enough that one RAS sweep is far from exact,
    # so every stage of the recurrence leaves a visible mark on the operator
    cfg = si.config_nested_square(n_base=4, n_ref=2, n_sub=16)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    J = fem.jacobian(cfg.u0, 10.0, geo, cfg.params)
    ras = krylov.RAS(J, fem.node_graph(geo), cfg.part, cfg.n_sub, cfg.overlap)
    Zn = krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n)
    tl = krylov.TwoLevel(J, ras, Zn)
    A = J.toarray()
    n = A.shape[0]
    Z = sp.kron(Zn, sp.identity(krylov.NC)).toarray()
    Q = Z @ np.linalg.solve(Z.T @ A @ Z, Z.T)          # R_0^T A_c^{-1} R_0
    M = _dense(ras.apply, n)
    return tl, A, M, Q, n


def _two_level_defects(apply):
    """Distances of the dense two-grid operator M2 = [apply] from (a) the
    error propagator (I - M A)(I - Q A)(I - M A) of the three-step recurrence
    and (b) the operator P5 = P4 + P3 - P3 A P4, P4 = P1 + P2 - P2 A P1 with
    P1 = P3 = M_RAS^{-1}, P2 = Q, as the substitution in Section 3.1 states."""
    tl, A, M, Q, n = _two_level_pieces()
    M2 = _dense(lambda r: apply(tl, r), n)
    I = np.eye(n)
    prop = (I - M @ A) @ (I - Q @ A) @ (I - M @ A)
    P4 = M + Q - Q @ A @ M
    P5 = P4 + M - M @ A @ P4
    scale = np.abs(M2).max()
    return (np.abs((I - M2 @ A) - prop).max(), np.abs(M2 - P5).max() / scale)


def test_two_level_operator_matches_the_three_step_recurrence():
    """Non-trivial nested coarse space (Z != I): the oracle's two-grid
    operator is the multiplicative fine-coarse-fine correction."""
    e_prop, e_p5 = _two_level_defects(krylov.TwoLevel.apply)
    assert e_prop <= 1e-10
    assert e_p5 <= 1e-12


def test_planted_two_level_mistakes_are_caught():
    """A dropped post-smoother, a dropped pre-smoother and an additive
    (residual not updated) coarse correction each break the pin above."""
    def no_post(tl, r):
        z1 = tl.ras.apply(r)
        return z1 + tl.coarse(r - tl.A @ z1)

    def no_pre(tl, r):
        z2 = tl.coarse(r)
        return z2 + tl.ras.apply(r - tl.A @ z2)

    def additive_coarse(tl, r):
        z1 = tl.ras.apply(r)
        z2 = z1 + tl.coarse(r)
        return z2 + tl.ras.apply(r - tl.A @ z2)

    for bad in (no_post, no_pre, additive_coarse):
        e_prop, e_p5 = _two_level_defects(bad)
        assert e_prop > 1e-2 and e_p5 > 1e-2, bad.__name__


def test_scalar_ras_pins():
    """One-compartment RAS (one unknown per node): a single subdomain is the
    exact inverse, and on a matrix decoupled along the partition the owner-
    restricted prolongation is exact while adding every copy is not."""
    cfg = si.config_small(nx=16)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    G = fem.node_graph(geo)
    Nbar = np.linspace(0.5, 1.5, len(geo.tri))
    A = (sp.diags(geo.mass) + 0.3 * newton._stiffness(geo, Nbar)).tocsr()
    b = np.random.default_rng(4).standard_normal(geo.n)
    x = spla.spsolve(A.tocsc(), b)
    one = krylov.RAS(A, G, np.zeros(geo.n, np.int32), 1, 0, bs=1)
    assert np.linalg.norm(one.apply(b) - x) <= 1e-12 * np.linalg.norm(x)
    Ac = A.tocoo()
    keep = cfg.part[Ac.row] == cfg.part[Ac.col]
    Ad = sp.coo_matrix((Ac.data[keep], (Ac.row[keep], Ac.col[keep])), shape=A.shape).tocsr()
    xd = spla.spsolve(Ad.tocsc(), b)
    ras = krylov.RAS(Ad, G, cfg.part, cfg.n_sub, 2, bs=1)
    assert np.linalg.norm(ras.apply(b) - xd) <= 1e-12 * np.linalg.norm(xd)
    assert np.linalg.norm(_asm_apply(ras, b) - xd) >= 1e-3 * np.linalg.norm(xd)


# ---------------------------------------------------------------------------
# Two-grid RAS-V2 (Section 3.2): coarse system solved by GMRES + coarse RAS
# ---------------------------------------------------------------------------
def _krylov_pieces(**kw):
    cfg = si.config_nested_square(n_base=4, n_ref=2, n_sub=16)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    J = fem.jacobian(cfg.u0, 10.0, geo, cfg.params)
    G = fem.node_graph(geo)
    ras = krylov.RAS(J, G, cfg.part, cfg.n_sub, cfg.overlap)
    Zn = krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n)
    tl = krylov.TwoLevel(J, ras, Zn)
    tk = krylov.TwoLevelKrylov(J, ras, Zn, G, cfg.part, cfg.n_sub, **kw)
    return cfg, J, Zn, G, tl, tk


def test_krylov_coarse_graph_is_the_coarse_triangulation():
    """On a nested grid the Galerkin coarse matrix couples exactly the
    coarse nodes joined by an edge of the coarse triangulation (a coarse hat
    function's support is its coarse star)."""
    nm = si.nested_square_mesh(4, 2)
    xy_c, tri_c = nm.levels[0]
    Zn = krylov.nested_interpolation(nm.parents[1:], len(xy_c))
    G = fem.node_graph(fem.Geometry(*nm.levels[-1]))
    C = krylov.coarse_graph(Zn, G)
    edges = set()
    for t in tri_c:
        for a, b in ((0, 1), (1, 2), (2, 0)):
            edges.add((min(t[a], t[b]), max(t[a], t[b])))
    Cu = sp.triu(C, 1).tocoo()
    assert set(zip(Cu.row.tolist(), Cu.col.tolist())) == edges


def test_krylov_coarse_partition_follows_the_coarse_nodes_own_fine_nodes():
    cfg, J, Zn, G, tl, tk = _krylov_pieces()
    cpart, nsc = krylov.coarse_partition(Zn, cfg.part, cfg.n_sub)
    Zc = Zn.tocsc()
    owners = []
    for I in range(Zn.shape[1]):
        col = Zc[:, I].toarray().ravel()
        own = np.nonzero(col == 1.0)[0]
        assert len(own) == 1          # the coarse node itself, on a nested grid
        owners.append(cfg.part[own[0]])
    used = sorted(set(owners))
    assert nsc == len(used)
    assert np.array_equal(cpart, [used.index(o) for o in owners])
    # merged groups: consecutive fine subdomain numbers
    cpart2, nsc2 = krylov.coarse_partition(Zn, cfg.part, cfg.n_sub, n_groups=4)
    assert nsc2 <= 4
    g = [o * 4 // cfg.n_sub for o in owners]
    assert np.array_equal(cpart2, np.searchsorted(sorted(set(g)), g))


def test_krylov_coarse_with_an_exact_inner_solve_is_the_two_grid_operator():
    """With the inner GMRES run to a tolerance near rounding, V2 applies the
    same operator as the direct coarse solve (pinned above against the
    three-step recurrence)."""
    cfg, J, Zn, G, tl, tk = _krylov_pieces(rtol=1e-15, atol=0.0, max_it=1000)
    r = np.random.default_rng(11).standard_normal(J.shape[0])
    a, b = tk.apply(r), tl.apply(r)
    assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)
    assert all(i["reason"] == "converged" for i in tk.infos)


def test_krylov_coarse_one_inner_iteration_has_its_closed_form():
    """One inner GMRES iteration from x0 = 0 returns alpha M_c r_c with
    alpha = <r_c, w> / <w, w>, w = A_c M_c r_c (the minimiser of the
    residual over span{M_c r_c}), M_c the coarse RAS."""
    cfg, J, Zn, G, tl, tk = _krylov_pieces(rtol=0.0, atol=0.0, max_it=1)
    r = np.random.default_rng(12).standard_normal(J.shape[0])
    rc = tk.Z.T @ r
    m = tk.ras_c.apply(rc)
    w = tk.Ac @ m
    alpha = np.dot(rc, w) / np.dot(w, w)
    got = tk.coarse(r)
    want = tk.Z @ (alpha * m)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    assert tk.infos[-1]["its"] == 1


def test_krylov_coarse_ras_is_restricted_on_the_coarse_graph():
    """The coarse RAS restricts with Boolean D_i: on a coarse matrix whose
    owner-to-owner couplings between subdomains are removed it is the exact
    inverse (as the fine-level pin above), which an additive (ASM) sum of
    the overlapping copies is not."""
    cfg, J, Zn, G, tl, tk = _krylov_pieces()
    cpart, nsc = krylov.coarse_partition(Zn, cfg.part, cfg.n_sub)
    Cg = krylov.coarse_graph(Zn, G)
    Ac = tk.Ac.tocoo()
    node_r, node_c = Ac.row // krylov.NC, Ac.col // krylov.NC
    keep = cpart[node_r] == cpart[node_c]
    Ad = sp.coo_matrix((Ac.data[keep], (Ac.row[keep], Ac.col[keep])), shape=Ac.shape).tocsr()
    ras_c = krylov.RAS(Ad, Cg, cpart, nsc, 1)
    b = np.random.default_rng(13).standard_normal(Ad.shape[0])
    x = spla.spsolve(Ad.tocsc(), b)
    assert np.linalg.norm(ras_c.apply(b) - x) <= 1e-10 * np.linalg.norm(x)
    asm = np.zeros_like(b)
    for idx, own, lu in ras_c.subs:
        asm[idx] += lu.solve(b[idx])
    assert np.linalg.norm(asm - x) > 1e-3 * np.linalg.norm(x)
