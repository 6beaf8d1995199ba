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
