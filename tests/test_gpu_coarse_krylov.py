"""Two-grid RAS-V2 and V3 on the GPU (coarse system solved by an inner GMRES
with RAS on the coarse graph, or with an aggregation-AMG V-cycle, Section
3.2) against the oracle's ``TwoLevelKrylov`` and its direct two-grid
operator, through the C ABI."""
import numpy as np
import pytest

import seird_inputs as si
from oracle import fem, krylov, newton

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402

DEV = "cuda"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def nested():
    cfg = si.config_nested_square(n_base=8, n_ref=2, n_sub=16)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    return cfg, prob, geo


def _harder(cfg):
    # dt = 1 with stronger diffusion: the coarse correction matters and the
    # inner solves need several iterations
    return si.Params(**{**cfg.params.__dict__, "nu": (0.05, 0.05, 0.02, 0.05, 0.0)})


def _system(cfg, prob, geo, seed, dt=1.0):
    p = _harder(cfg)
    prob.set_params(p)
    rng = np.random.default_rng(seed)
    u = cfg.u0 * rng.uniform(0.8, 1.2, cfg.u0.shape) + rng.uniform(0, 0.01, cfg.u0.shape)
    vals = prob.jacobian(T(u), dt)
    Jo = fem.jacobian(u, dt, geo, p)
    G = fem.node_graph(geo)
    ras = krylov.RAS(Jo, G, cfg.part, cfg.n_sub, cfg.overlap)
    Zn = krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n)
    return vals, Jo, G, ras, Zn


def _precond(cfg, prob, vals, **kw):
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    pc.set_coarse_krylov(**kw)
    pc.setup(vals)
    return pc


def test_exact_inner_solve_gives_the_direct_two_grid_operator(nested):
    cfg, prob, geo = nested
    try:
        vals, Jo, G, ras, Zn = _system(cfg, prob, geo, 21)
        pc = _precond(cfg, prob, vals, rtol=1e-14, atol=0.0, max_it=400)
        r = np.random.default_rng(1).standard_normal(5 * cfg.n)
        z = H(pc.apply(T(r)))
        assert relerr(z, krylov.TwoLevel(Jo, ras, Zn).apply(r)) < 1e-9
        st = pc.coarse_krylov_stats()
        _, nsc = krylov.coarse_partition(Zn, cfg.part, cfg.n_sub)
        assert st["solves"] == 1 and st["unconverged"] == 0 and st["its"] > 1
        assert st["coarse_subdomains"] == nsc
    finally:
        prob.set_params(cfg.params)


@pytest.mark.parametrize("its,groups", [(1, 0), (3, 0), (8, 0), (5, 4)])
def test_capped_inner_solve_matches_oracle(nested, its, groups):
    """rtol = atol = 0: both inner GMRES run exactly `its` iterations, so the
    GPU operator and the oracle's are the same polynomial in the coarse
    RAS-preconditioned coarse matrix."""
    cfg, prob, geo = nested
    try:
        vals, Jo, G, ras, Zn = _system(cfg, prob, geo, 22)
        pc = _precond(cfg, prob, vals, n_sub=groups, rtol=0.0, atol=0.0, max_it=its)
        tk = krylov.TwoLevelKrylov(Jo, ras, Zn, G, cfg.part, cfg.n_sub, n_groups=groups,
                                   rtol=0.0, atol=0.0, max_it=its)
        r = np.random.default_rng(2).standard_normal(5 * cfg.n)
        assert relerr(H(pc.apply(T(r))), tk.apply(r)) < 1e-10
        st = pc.coarse_krylov_stats(reset=True)
        assert st["solves"] == 1 and st["its"] == its and st["unconverged"] == 1
        assert st["coarse_subdomains"] == tk.n_coarse_sub
    finally:
        prob.set_params(cfg.params)


def test_outer_gmres_matches_oracle_flexible_gmres(nested):
    cfg, prob, geo = nested
    try:
        vals, Jo, G, ras, Zn = _system(cfg, prob, geo, 23)
        pc = _precond(cfg, prob, vals)  # the paper's settings: rtol 1e-5, 100 inner its
        tk = krylov.TwoLevelKrylov(Jo, ras, Zn, G, cfg.part, cfg.n_sub)
        b = np.random.default_rng(3).standard_normal(5 * cfg.n)
        for rtol in (1e-5, 1e-10):
            x, st = sk.gmres(prob, pc, vals, T(b), rtol=rtol)
            xo, io = krylov.gmres(lambda v: Jo @ v, b, tk.apply, rtol=rtol)
            assert st["reason"] == 1 and io["reason"] == "converged"
            assert abs(st["its"] - io["its"]) <= 1, (st, io)
            assert np.linalg.norm(Jo @ H(x) - b) <= 1.01 * rtol * np.linalg.norm(b)
        ks = pc.coarse_krylov_stats()
        assert ks["solves"] >= 2 and ks["unconverged"] == 0
    finally:
        prob.set_params(cfg.params)


def test_newton_steps_with_krylov_coarse_reach_the_oracle_root(nested):
    cfg, prob, geo = nested
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    pc.set_coarse_krylov()
    u = T(cfg.u0.copy())
    uo = cfg.u0.copy()
    for _ in range(3):
        sk.step(prob, pc, u, cfg.dt, tol=1e-13, rtol=1e-9)
        uo, _ = newton.newton_step(uo, cfg.dt, geo, cfg.params, tol=1e-14)
    ug = H(u)
    for c in range(5):
        assert np.abs(ug[:, c] - uo[:, c]).max() <= 1e-8 * max(np.abs(uo[:, c]).max(), 1e-30), c
    assert pc.coarse_krylov_stats()["solves"] > 0


def test_krylov_coarse_misuse_is_reported(nested):
    cfg, prob, geo = nested
    vals = prob.jacobian(T(cfg.u0), cfg.dt)
    pc = _precond(cfg, prob, vals)
    r = T(np.random.default_rng(4).standard_normal(5 * cfg.n))
    with pytest.raises(sk.SeirdError) as e:
        pc.apply(r, transpose=True)
    assert e.value.code == -1
    pc.set_coarse_solver(0)  # direct again: needs a setup first
    with pytest.raises(sk.SeirdError) as e:
        pc.apply(r)
    assert e.value.code == -1
    pc.setup(vals)
    z0 = H(pc.apply(r))
    pc.set_coarse_solver(2)
    pc.setup(vals)
    z2 = H(pc.apply(r))
    assert relerr(z2, z0) < 1e-3  # inner rtol 1e-5: close to the direct solve
    one = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    with pytest.raises(sk.SeirdError) as e:
        one.set_coarse_krylov()
    assert e.value.code == -1
    with pytest.raises(sk.SeirdError):
        pc.set_coarse_krylov(restart=0)


# --------------------------------------------------------------------------
# V3: inner GMRES preconditioned by the aggregation AMG V-cycle
# --------------------------------------------------------------------------
AMG = dict(max_coarse=4, nu=1, omega=2.0 / 3.0)  # levels of 81, 9 and 1 nodes


def _precond_amg(cfg, prob, vals, **kw):
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    pc.set_coarse_amg(**{**AMG, **kw})
    pc.setup(vals)
    return pc


def test_v3_exact_inner_solve_gives_the_direct_two_grid_operator(nested):
    cfg, prob, geo = nested
    try:
        vals, Jo, G, ras, Zn = _system(cfg, prob, geo, 31)
        pc = _precond_amg(cfg, prob, vals, rtol=1e-14, atol=0.0, max_it=400)
        r = np.random.default_rng(6).standard_normal(5 * cfg.n)
        assert relerr(H(pc.apply(T(r))), krylov.TwoLevel(Jo, ras, Zn).apply(r)) < 1e-9
        st = pc.coarse_krylov_stats()
        tk = krylov.TwoLevelKrylov(Jo, ras, Zn, G, cfg.part, cfg.n_sub, inner="amg", amg=AMG)
        assert st["amg_levels"] == tk.amg.levels >= 3
        assert st["amg_last_nodes"] == tk.amg.A[-1].shape[0] // 5
        assert st["unconverged"] == 0
    finally:
        prob.set_params(cfg.params)


@pytest.mark.parametrize("its,nu", [(1, 1), (4, 1), (3, 2)])
def test_v3_capped_inner_solve_matches_oracle(nested, its, nu):
    """The same aggregates, smoothing and last-level solve as the oracle's
    AMG: the capped inner solves give the same operator."""
    cfg, prob, geo = nested
    try:
        vals, Jo, G, ras, Zn = _system(cfg, prob, geo, 32)
        pc = _precond_amg(cfg, prob, vals, nu=nu, rtol=0.0, atol=0.0, max_it=its)
        tk = krylov.TwoLevelKrylov(Jo, ras, Zn, G, cfg.part, cfg.n_sub, inner="amg", amg={**AMG, "nu": nu},
                                   rtol=0.0, atol=0.0, max_it=its)
        r = np.random.default_rng(7).standard_normal(5 * cfg.n)
        assert relerr(H(pc.apply(T(r))), tk.apply(r)) < 1e-10
    finally:
        prob.set_params(cfg.params)


def test_v3_outer_gmres_matches_oracle(nested):
    cfg, prob, geo = nested
    try:
        vals, Jo, G, ras, Zn = _system(cfg, prob, geo, 33)
        pc = _precond_amg(cfg, prob, vals)
        tk = krylov.TwoLevelKrylov(Jo, ras, Zn, G, cfg.part, cfg.n_sub, inner="amg", amg=AMG)
        b = np.random.default_rng(8).standard_normal(5 * cfg.n)
        x, st = sk.gmres(prob, pc, vals, T(b), rtol=1e-8)
        xo, io = krylov.gmres(lambda v: Jo @ v, b, tk.apply, rtol=1e-8)
        assert st["reason"] == 1 and io["reason"] == "converged"
        assert abs(st["its"] - io["its"]) <= 1, (st, io)
        assert np.linalg.norm(Jo @ H(x) - b) <= 1.01e-8 * np.linalg.norm(b)
    finally:
        prob.set_params(cfg.params)


def test_v3_newton_steps_reach_the_oracle_root(nested):
    cfg, prob, geo = nested
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    pc.set_coarse_amg()
    u = T(cfg.u0.copy())
    uo = cfg.u0.copy()
    for _ in range(3):
        sk.step(prob, pc, u, cfg.dt, tol=1e-13, rtol=1e-9)
        uo, _ = newton.newton_step(uo, cfg.dt, geo, cfg.params, tol=1e-14)
    ug = H(u)
    for c in range(5):
        assert np.abs(ug[:, c] - uo[:, c]).max() <= 1e-8 * max(np.abs(uo[:, c]).max(), 1e-30), c
    with pytest.raises(sk.SeirdError):
        pc.set_coarse_solver(2)  # no Krylov-RAS coarse solver on this preconditioner
    with pytest.raises(sk.SeirdError):
        pc.set_coarse_amg(omega=2.5)
