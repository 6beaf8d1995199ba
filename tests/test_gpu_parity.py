"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Floating-point tolerances are normwise relative; the
assembly kernels differ from the oracle only in summation order
(|err| <~ 1e-15 * condition), the solves are compared at the tolerance the
solver was asked for."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

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


def jac_to_scipy(prob, vals):
    """Decode the library's node-block Jacobian layout into scipy CSR."""
    v = H(vals)
    n = prob.n
    diag = v[:25 * n].reshape(n, 5, 5)
    off = v[25 * n:].reshape(-1, 10)
    rp, col = prob.pattern()
    rows, cols, data = [], [], []
    node = np.arange(n)
    for c in range(5):
        for cp in range(5):
            rows.append(5 * node + c)
            cols.append(5 * node + cp)
            data.append(diag[:, c, cp])
    src = np.repeat(np.arange(n), np.diff(rp))
    for c in range(5):
        for cp in range(5):
            rows.append(5 * src + c)
            cols.append(5 * col + cp)
            data.append(off[:, 5 + c] + (off[:, c] if c == cp else 0.0))
    return sp.coo_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(5 * n, 5 * n)).tocsr()


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _state(cfg, seed):
    rng = np.random.default_rng(seed)
    return cfg.u0 * rng.uniform(0.8, 1.2, cfg.u0.shape) + rng.uniform(0, 0.01, cfg.u0.shape)


@pytest.fixture(scope="module")
def small():
    cfg = si.config_small()
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    return cfg, prob, geo


def test_residual_matches_oracle(small):
    cfg, prob, geo = small
    p = si.Params(**{**cfg.params.__dict__, "nu": (1e-3, 2e-3, 5e-4, 1e-3, 3e-4),
                     "alpha": 0.01, "mu": 0.005})
    prob.set_params(p)
    try:
        for seed in range(3):
            u = _state(cfg, seed)
            up = _state(cfg, seed + 10)
            src = np.random.default_rng(seed).standard_normal(u.shape)
            g = np.random.default_rng(seed + 5).uniform(0.5, 1.5, cfg.n)
            prob.set_beta_field(T(g))
            F = H(prob.residual(T(u), T(up), 0.37, src=T(src)))
            Fo = fem.residual(u, up, 0.37, geo, p, g, src)
            assert relerr(F, Fo) < 1e-13
            assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
        prob.set_beta_field(None)
    finally:
        prob.set_params(cfg.params)


def test_jacobian_matches_oracle_entrywise(small):
    cfg, prob, geo = small
    p = si.Params(**{**cfg.params.__dict__, "nu": (1e-3, 2e-3, 5e-4, 1e-3, 3e-4),
                     "alpha": 0.01, "mu": 0.005})
    prob.set_params(p)
    try:
        u = _state(cfg, 3)
        J = jac_to_scipy(prob, prob.jacobian(T(u), 0.21))
        Jo = fem.jacobian(u, 0.21, geo, p)
        D = (J - Jo).tocoo()
        assert np.abs(D.data).max(initial=0) <= 1e-13 * np.abs(Jo.data).max()
    finally:
        prob.set_params(cfg.params)


def test_spmv_and_transpose_match_scipy(small):
    cfg, prob, geo = small
    u = _state(cfg, 4)
    vals = prob.jacobian(T(u), cfg.dt)
    Jo = fem.jacobian(u, cfg.dt, geo, cfg.params)
    x = np.random.default_rng(0).standard_normal(5 * cfg.n)
    y = H(prob.spmv(vals, T(x)))
    yt = H(prob.spmv(vals, T(x), transpose=True))
    assert relerr(y, Jo @ x) < 1e-14
    assert relerr(yt, Jo.T @ x) < 1e-14


def test_one_subdomain_ras_is_the_exact_inverse(small):
    cfg, prob, geo = small
    u = _state(cfg, 5)
    vals = prob.jacobian(T(u), cfg.dt)
    pc = sk.Precond(prob, np.zeros(cfg.n, np.int32), 1, 0)
    pc.setup(vals)
    Jo = fem.jacobian(u, cfg.dt, geo, cfg.params).tocsc()
    r = np.random.default_rng(1).standard_normal(5 * cfg.n)
    z = H(pc.apply(T(r)))
    zo = spla.spsolve(Jo, r)
    assert relerr(z, zo) < 1e-10
    zt = H(pc.apply(T(r), transpose=True))
    assert relerr(zt, spla.spsolve(Jo.T.tocsc(), r)) < 1e-10


@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("overlap", [1, 2])
def test_ras_apply_matches_oracle(small, tile, overlap):
    cfg, prob, geo = small
    u = _state(cfg, 6)
    vals = prob.jacobian(T(u), cfg.dt)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, overlap, tile=tile)
    pc.setup(vals)
    Jo = fem.jacobian(u, cfg.dt, geo, cfg.params)
    ras = krylov.RAS(Jo, fem.node_graph(geo), cfg.part, cfg.n_sub, overlap)
    r = np.random.default_rng(2).standard_normal(5 * cfg.n)
    assert relerr(H(pc.apply(T(r))), ras.apply(r)) < 1e-11
    assert relerr(H(pc.apply(T(r), transpose=True)), ras.apply_T(r)) < 1e-11


def _wheel_mesh(rings=8, spokes=24):
    """Polar mesh: a centre node of degree `spokes` inside rings of `spokes`
    nodes (every other node has degree <= 6); triangles counter-clockwise."""
    xy = [(0.0, 0.0)]
    for r in range(1, rings + 1):
        for k in range(spokes):
            t = 2 * np.pi * k / spokes
            xy.append((r * np.cos(t), r * np.sin(t)))
    node = lambda r, k: 1 + (r - 1) * spokes + k % spokes  # noqa: E731
    tri = [(0, node(1, k), node(1, k + 1)) for k in range(spokes)]
    for r in range(1, rings):
        for k in range(spokes):
            a, b, c, d = node(r, k), node(r, k + 1), node(r + 1, k + 1), node(r + 1, k)
            tri += [(a, c, b), (a, d, c)]
    return np.array(xy), np.array(tri, dtype=np.int32)


@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("overlap", [1, 2])
def test_ras_apply_with_a_high_degree_node(small, tile, overlap):
    """A node with more blocks than the extraction holds in registers (its
    rows search the entry list in memory) still gives the oracle's RAS."""
    cfg = small[0]
    xy, tri = _wheel_mesh()
    n = len(xy)
    part = (((np.arctan2(xy[:, 1], xy[:, 0]) + np.pi) / (2 * np.pi) * 4).astype(np.int32)) % 4
    prob = sk.Problem(xy, tri, cfg.params)
    geo = fem.Geometry(xy, tri)
    rng = np.random.default_rng(11)
    u = np.abs(cfg.u0[:n]) * rng.uniform(0.8, 1.2, (n, 5)) + rng.uniform(0.01, 0.1, (n, 5))
    vals = prob.jacobian(T(u), cfg.dt)
    pc = sk.Precond(prob, part, 4, overlap, tile=tile)
    pc.setup(vals)
    Jo = fem.jacobian(u, cfg.dt, geo, cfg.params)
    ras = krylov.RAS(Jo, fem.node_graph(geo), part, 4, overlap)
    r = rng.standard_normal(5 * n)
    assert relerr(H(pc.apply(T(r))), ras.apply(r)) < 1e-11
    assert relerr(H(pc.apply(T(r), transpose=True)), ras.apply_T(r)) < 1e-11


@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (2, 3e-2)])
def test_reduced_precision_factors_stay_close(small, prec, tol):
    cfg, prob, geo = small
    u = _state(cfg, 7)
    vals = prob.jacobian(T(u), cfg.dt)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, 1, factor_prec=prec)
    pc.setup(vals)
    Jo = fem.jacobian(u, cfg.dt, geo, cfg.params)
    ras = krylov.RAS(Jo, fem.node_graph(geo), cfg.part, cfg.n_sub, 1)
    r = np.random.default_rng(3).standard_normal(5 * cfg.n)
    assert relerr(H(pc.apply(T(r))), ras.apply(r)) < tol


@pytest.fixture(scope="module")
def nested():
    cfg = si.config_nested_square(n_base=8, n_ref=2, n_sub=16)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    return cfg, prob, geo


def test_two_level_apply_matches_oracle(nested):
    cfg, prob, geo = nested
    u = _state(cfg, 8)
    vals = prob.jacobian(T(u), cfg.dt)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap,
                    coarse=(cfg.coarse_parents, cfg.coarse_n))
    pc.setup(vals)
    Jo = fem.jacobian(u, cfg.dt, geo, cfg.params)
    ras = krylov.RAS(Jo, fem.node_graph(geo), cfg.part, cfg.n_sub, cfg.overlap)
    tl = krylov.TwoLevel(Jo, ras, krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n))
    r = np.random.default_rng(4).standard_normal(5 * cfg.n)
    assert relerr(H(pc.apply(T(r))), tl.apply(r)) < 1e-10
    assert relerr(H(pc.apply(T(r), transpose=True)), tl.apply_T(r)) < 1e-10


def _bigger_dt(cfg):
    # a harder linear system than the configuration's own, so that GMRES
    # needs more than a couple of iterations
    return si.Params(**{**cfg.params.__dict__, "nu": (0.05, 0.05, 0.02, 0.05, 0.0)})


@pytest.mark.parametrize("two_level", [False, True])
def test_gmres_iterations_and_solution_match_oracle(nested, two_level):
    cfg, prob, geo = nested
    p = _bigger_dt(cfg)
    prob.set_params(p)
    try:
        u = _state(cfg, 9)
        vals = prob.jacobian(T(u), 1.0)
        coarse = (cfg.coarse_parents, cfg.coarse_n) if two_level else None
        pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse)
        pc.setup(vals)
        Jo = fem.jacobian(u, 1.0, geo, p)
        ras = krylov.RAS(Jo, fem.node_graph(geo), cfg.part, cfg.n_sub, cfg.overlap)
        M = ras if not two_level else krylov.TwoLevel(
            Jo, ras, krylov.nested_interpolation(cfg.coarse_parents, cfg.coarse_n))
        b = np.random.default_rng(5).standard_normal(5 * cfg.n)
        for rtol, restart in ((1e-5, 30), (1e-10, 5)):
            x, st = sk.gmres(prob, pc, vals, T(b), rtol=rtol, restart=restart)
            xo, io = krylov.gmres(lambda v: Jo @ v, b, M.apply, rtol=rtol, restart=restart)
            assert st["reason"] == 1 and io["reason"] == "converged"
            assert abs(st["its"] - io["its"]) <= 1, (st, io)
            assert np.linalg.norm(Jo @ H(x) - b) <= 1.01 * rtol * np.linalg.norm(b)
        # transposed solve
        x, st = sk.gmres(prob, pc, vals, T(b), transpose=True, rtol=1e-10)
        assert np.linalg.norm(Jo.T @ H(x) - b) <= 1.01e-10 * np.linalg.norm(b)
    finally:
        prob.set_params(cfg.params)


def _field_errors(ug, uo):
    """Per-field normwise errors: relative to the field itself and relative
    to the whole state (the scale of the Newton stopping test)."""
    scale = np.linalg.norm(uo)
    own, glob = [], []
    for c in range(5):
        d = np.linalg.norm(ug[:, c] - uo[:, c])
        glob.append(d / scale)
        nref = np.linalg.norm(uo[:, c])
        own.append(d / nref if nref > 0 else (0.0 if d == 0 else np.inf))
    return np.array(own), np.array(glob)


def test_small_config_ten_steps_match_oracle(small):
    """The small configuration end to end at its own tolerances (Newton
    1e-10, GMRES rtol 1e-5): every field within 1e-8 of the oracle's
    direct-solve root relative to the state scale, the GPU state solves the
    oracle's residual to the tolerance, population is conserved."""
    cfg, prob, geo = small
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    u = T(cfg.u0.copy())
    uo = cfg.u0.copy()
    P0 = fem.total_population(uo, geo)
    for n in range(cfg.steps):
        uprev = H(u).copy()
        st = sk.step(prob, pc, u, cfg.dt, tol=cfg.newton_tol)
        uo, info = newton.newton_step(uo, cfg.dt, geo, cfg.params, tol=1e-13)
        ug = H(u)
        own, glob = _field_errors(ug, uo)
        assert glob.max() < 1e-8, (n, glob)
        assert np.abs(ug - uo).max() <= 1e-8 * np.abs(uo).max()
        Fo = fem.residual(ug, uprev, cfg.dt, geo, cfg.params)
        assert np.linalg.norm(Fo) <= 1.01 * cfg.newton_tol * np.linalg.norm(geo.mass[:, None] * uprev)
        assert abs(fem.total_population(ug, geo) - P0) <= 1e-10 * P0
        assert st["res_hist"][-1] <= cfg.newton_tol


def test_small_config_tight_solve_matches_every_field(small):
    """Tight solver settings (Newton 1e-13, GMRES rtol 1e-9): every field,
    including the small exposed/recovered/deceased densities, within 1e-8
    relative of the oracle root, normwise and in max norm."""
    cfg, prob, geo = small
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    u = T(cfg.u0.copy())
    uo = cfg.u0.copy()
    for n in range(cfg.steps):
        sk.step(prob, pc, u, cfg.dt, tol=1e-13, rtol=1e-9)
        uo, _ = newton.newton_step(uo, cfg.dt, geo, cfg.params, tol=1e-14)
        ug = H(u)
        own, _ = _field_errors(ug, uo)
        assert own.max() < 1e-8, (n, own)
        for c in range(5):
            m = np.abs(uo[:, c]).max()
            assert np.abs(ug[:, c] - uo[:, c]).max() <= 1e-8 * m, (n, c)


def test_lagged_preconditioner_reaches_the_same_root(small):
    """Reusing one preconditioner setup for every Newton iteration of a step
    changes GMRES iteration counts only: the root matches the oracle."""
    cfg, prob, geo = small
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    u = T(cfg.u0.copy())
    uo = cfg.u0.copy()
    for n in range(3):
        st = sk.step(prob, pc, u, cfg.dt, tol=1e-13, rtol=1e-9, pc_reuse=100)
        assert st["pc_setups"] == 1
        uo, _ = newton.newton_step(uo, cfg.dt, geo, cfg.params, tol=1e-14)
    own, _ = _field_errors(H(u), uo)
    assert own.max() < 1e-8, own


def test_two_level_steps_match_oracle(nested):
    cfg, prob, geo = nested
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap,
                    coarse=(cfg.coarse_parents, cfg.coarse_n))
    u = T(cfg.u0.copy())
    uo = cfg.u0.copy()
    for n in range(3):
        sk.step(prob, pc, u, cfg.dt, tol=1e-13, rtol=1e-9)
        uo, _ = newton.newton_step(uo, cfg.dt, geo, cfg.params, tol=1e-14)
    own, _ = _field_errors(H(u), uo)
    assert own.max() < 1e-8, own


def test_steps_are_bitwise_reproducible(small):
    cfg, prob, geo = small
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    outs = []
    for _ in range(2):
        u = T(cfg.u0.copy())
        for n in range(2):
            sk.step(prob, pc, u, cfg.dt, tol=cfg.newton_tol)
        outs.append(H(u))
    assert np.array_equal(outs[0], outs[1])


def test_error_paths_return_status_codes(small):
    cfg, prob, geo = small
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    u = cfg.u0.copy()
    u[7, 2] = np.nan
    with pytest.raises(sk.SeirdError) as e:
        sk.step(prob, pc, T(u), cfg.dt)
    assert e.value.code == -4
    u = cfg.u0.copy()
    u[9, :] = 0.0
    with pytest.raises(sk.SeirdError) as e:
        sk.step(prob, pc, T(u), cfg.dt)
    assert e.value.code == -9
    with pytest.raises(sk.SeirdError) as e:
        sk.step(prob, pc, T(cfg.u0.copy()), cfg.dt, tol=1e-30, max_it=1)
    assert e.value.code == -7
    bad = cfg.tri.copy()
    bad[0] = [0, 1, 2]  # collinear nodes on the bottom edge
    with pytest.raises(sk.SeirdError) as e:
        sk.Problem(cfg.xy, bad, cfg.params)
    assert e.value.code == -2
    with pytest.raises(sk.SeirdError) as e:
        sk.Precond(prob, np.full(cfg.n, 99, np.int32), 4, 1)
    assert e.value.code == -1


def test_kept_setups_across_steps_reach_the_same_states():
    """A setup kept for two later steps (pc_keep_steps) gives the states of
    one setup per step within the Newton tolerance, with fewer setups; a
    change of dt takes a fresh setup."""
    cfg = si.config_small()
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pa = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    pb = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    ua = T(cfg.u0)
    ub = T(cfg.u0)
    kw = dict(tol=1e-12, rtol=1e-10, pc_reuse=100)
    setups = []
    for _ in range(cfg.steps):
        sk.step(prob, pa, ua, cfg.dt, **kw)
        setups.append(sk.step(prob, pb, ub, cfg.dt, pc_keep_steps=2, **kw)["pc_setups"])
    # one setup serves three steps unless its GMRES count grows past its budget
    assert setups[0] == 1 and setups[1] == 0 and sum(setups) <= (cfg.steps + 2) // 3 + 2, setups
    assert relerr(H(ub), H(ua)) < 1e-9
    st = sk.step(prob, pb, ub, 0.5 * cfg.dt, pc_keep_steps=2, **kw)
    assert st["pc_setups"] == 1
