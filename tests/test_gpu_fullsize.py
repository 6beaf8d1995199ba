"""Parity at the realistic workload's full size (about 1.01M nodes, 5.04M
unknowns; two-grid RAS with 1024 subdomains, overlap 2) in the launch
configuration the benchmark times.

The oracle cannot assemble or factor the whole 5M-unknown system quickly,
so it checks outputs it can compute one by one:
* residual rows everywhere (vectorised numpy) and Jacobian rows of sampled
  nodes (oracle Jacobian of the triangles incident to the sample, which is
  exact for the sampled rows);
* the RAS output on the owned nodes of sampled subdomains (the oracle's
  exact local solve of R_i A R_i^T);
and properties that hold at any size for a full implicit step: the oracle
residual of the GPU state is below the tolerance, population is
conserved, densities stay positive."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import seird_inputs as si
from oracle import fem, krylov

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402


@pytest.fixture(scope="module")
def big():
    cfg = si.config_realistic()
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    return cfg, prob, geo


def _incident(tri, nodes):
    mask = np.zeros(tri.max() + 1, dtype=bool)
    mask[nodes] = True
    return tri[mask[tri].any(1)]


def test_fullsize_residual_and_sampled_jacobian_rows(big):
    cfg, prob, geo = big
    rng = np.random.default_rng(0)
    u = cfg.u0 * rng.uniform(0.9, 1.1, cfg.u0.shape)
    F = prob.residual(torch.tensor(u, device="cuda"), torch.tensor(cfg.u0, device="cuda"), cfg.dt)
    Fo = fem.residual(u, cfg.u0, cfg.dt, geo, cfg.params)
    Fg = F.cpu().numpy()
    assert np.linalg.norm(Fg - Fo) <= 1e-13 * np.linalg.norm(Fo)
    # Jacobian rows of 2000 sampled nodes
    vals = prob.jacobian(torch.tensor(u, device="cuda"), cfg.dt)
    x = rng.standard_normal(5 * cfg.n)
    y = prob.spmv(vals, torch.tensor(x, device="cuda")).cpu().numpy()
    sample = rng.choice(cfg.n, 2000, replace=False)
    sub = fem.Geometry(cfg.xy, _incident(cfg.tri, sample))
    Js = fem.jacobian(u, cfg.dt, sub, cfg.params)
    rows = (5 * sample[:, None] + np.arange(5)[None, :]).ravel()
    yo = Js[rows] @ x
    assert np.linalg.norm(y[rows] - yo) <= 1e-13 * np.linalg.norm(yo)


def test_fullsize_ras_on_sampled_subdomains(big):
    cfg, prob, geo = big
    rng = np.random.default_rng(1)
    u = cfg.u0
    vals = prob.jacobian(torch.tensor(u, device="cuda"), cfg.dt)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)  # one-level: RAS alone
    pc.setup(vals)
    r = rng.standard_normal(5 * cfg.n)
    z = pc.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    G = fem.node_graph(geo)
    for s in rng.choice(cfg.n_sub, 6, replace=False):
        owned = np.nonzero(cfg.part == s)[0]
        nodes = krylov.grow_overlap(G, owned, cfg.overlap)
        subg = fem.Geometry(cfg.xy, _incident(cfg.tri, nodes))
        Js = fem.jacobian(u, cfg.dt, subg, cfg.params).tocsr()
        idx = krylov.unknowns_of(nodes)
        Ai = Js[idx][:, idx].tocsc()
        zi = spla.splu(Ai).solve(r[idx])
        own = np.repeat(cfg.part[nodes] == s, 5)
        zo = zi[own]
        zg = z[idx[own]]
        assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo), s


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_fullsize_step_solves_the_oracle_residual(big, prec):
    cfg, prob, geo = big
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, factor_prec=prec,
                    coarse=(cfg.coarse_parents, cfg.coarse_n))
    u = torch.tensor(cfg.u0, device="cuda")
    st = sk.step(prob, pc, u, cfg.dt, tol=cfg.newton_tol, pc_reuse=100)
    ug = u.cpu().numpy()
    Fo = fem.residual(ug, cfg.u0, cfg.dt, geo, cfg.params)
    scale = np.linalg.norm(geo.mass[:, None] * cfg.u0)
    assert np.linalg.norm(Fo) <= 1.01 * cfg.newton_tol * scale, st
    P0 = fem.total_population(cfg.u0, geo)
    assert abs(fem.total_population(ug, geo) - P0) <= 1e-9 * P0
    assert ug[:, 0].min() > 0 and ug.sum(1).min() > 0


def test_fullsize_ensemble_step():
    """The 48-instance ensemble (about 9.3M nodes, 46.7M unknowns) in the
    benchmark's configuration (FP32 factors, lagged setup): on sampled
    instances the oracle residual of the GPU state is below the tolerance;
    on all instances population is conserved and densities stay positive."""
    bc = si.config_batch()
    inst = bc.instances
    b = sk.Batch([(c.xy, c.tri, c.params, c.part, c.n_sub) for c in inst],
                 overlap=bc.overlap, factor_prec=1)
    u = torch.tensor(np.concatenate([c.u0 for c in inst]), device="cuda")
    tol = inst[0].newton_tol
    per = b.step(u, bc.dt, tol=tol, pc_reuse=100)
    print("ensemble step: newton", [p["newton_its"] for p in per], "gmres",
          [sum(p["gmres_its"]) for p in per], "halvings", [p["backtracks"] for p in per], flush=True)
    ub = u.cpu().numpy()
    off = b.node_offsets
    sizes = [c.n for c in inst]
    rng = np.random.default_rng(3)
    sample = {int(np.argmin(sizes)), int(np.argmax(sizes)), int(rng.integers(len(inst)))}
    for k, c in enumerate(inst):
        uk = ub[off[k]:off[k + 1]]
        geo = fem.Geometry(c.xy, c.tri)
        P0 = fem.total_population(c.u0, geo)
        assert abs(fem.total_population(uk, geo) - P0) <= 1e-9 * P0, k
        assert uk[:, 0].min() > 0 and uk.sum(1).min() > 0, k
        assert per[k]["res_hist"][-1] <= tol, k
        if k in sample:
            Fo = fem.residual(uk, c.u0, c.dt, geo, c.params)
            scale = np.linalg.norm(geo.mass[:, None] * c.u0)
            assert np.linalg.norm(Fo) <= 1.01 * tol * scale, (k, per[k])


def test_fullsize_differentiation_gradient_matches_finite_differences():
    """The differentiation workload's mesh (about 2M nodes, 10M unknowns,
    two-grid RAS with 2048 subdomains), cut to 3 daily steps: the adjoint
    gradient with respect to the transmission field agrees with central
    finite differences (h = 1e-6) to 1e-5 relative in two directions; the
    observation regions and the truth field are the workload's (40 Voronoi
    regions, perturbed field).  At 10M unknowns the forward solves stop at a
    scaled residual of 1e-12, so J carries relative noise of about that
    order; the directions are smooth random fields (signed Gaussian bumps,
    max-norm 1), for which the derivative is of the size of J and the
    difference quotient resolves it."""
    cfg = si.config_differentiation()
    steps = 3
    region = si.voronoi_regions(cfg.xy, 40, seed=8)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    kw = dict(tol=1e-12, rtol=1e-11)

    def run(g):
        prob.set_beta_field(torch.tensor(g, device="cuda"))
        u = torch.tensor(cfg.u0, device="cuda")
        return sk.forward_record(prob, pc, u, steps, cfg.dt, region, 40, ckpt_every=2, **kw)

    truth = run(si.bump_field(cfg.xy, seed=7)).cpu().numpy()
    g0 = np.ones(cfg.n)
    c = run(g0)
    gg, _, st = sk.adjoint(prob, pc, 2 * (c - torch.tensor(truth, device="cuda")), rtol=1e-10)
    gg = gg.cpu().numpy()

    def J(g):
        return float(((run(g).cpu().numpy() - truth) ** 2).sum())

    h = 1e-6
    for seed in (9, 10):
        d = si.bump_field(cfg.xy, seed=seed, amp=1.0) - 1.0
        d /= np.abs(d).max()
        fd = (J(g0 + h * d) - J(g0 - h * d)) / (2 * h)
        assert fd == pytest.approx(gg @ d, rel=1e-5), (fd, gg @ d, st)


def test_fullsize_thirty_steps_each_solve_the_oracle_residual(big):
    """The workload's 30 daily steps (FP64 factors, the benchmark's
    launch configuration): after every step the oracle residual of the GPU
    state, with the previous GPU state as u^n, is below the tolerance;
    population is conserved throughout."""
    cfg, prob, geo = big
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    u = torch.tensor(cfg.u0, device="cuda")
    prev = cfg.u0.copy()
    P0 = fem.total_population(cfg.u0, geo)
    for k in range(cfg.steps):
        st = sk.step(prob, pc, u, cfg.dt, tol=cfg.newton_tol, pc_reuse=100)
        ug = u.cpu().numpy()
        Fo = fem.residual(ug, prev, cfg.dt, geo, cfg.params)
        scale = np.linalg.norm(geo.mass[:, None] * prev)
        assert np.linalg.norm(Fo) <= 1.01 * cfg.newton_tol * scale, (k, st)
        assert abs(fem.total_population(ug, geo) - P0) <= 1e-9 * P0, k
        prev = ug


def test_differentiation_recipe_sixty_steps_twenty_directions():
    """The differentiation workload's recipe at the nested size (same seed
    and polygon, about 31k nodes, 32 subdomains, two-grid RAS) over its full
    60 daily steps with checkpoints every 10 and its 40 Voronoi regions and
    perturbed truth field: the adjoint gradient with respect to the
    transmission field agrees with central finite differences (h = 1e-6) to
    1e-5 relative in 20 smooth random directions, and the gradients with
    respect to the five diffusion coefficients in all five."""
    cfg = si.config_differentiation(n_base=122, n_ref=4, n_sub=32)
    steps = cfg.steps
    assert steps == 60
    region = si.voronoi_regions(cfg.xy, 40, seed=8)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=(cfg.coarse_parents, cfg.coarse_n))
    # one preconditioner setup per step (the root does not depend on it)
    kw = dict(tol=1e-12, rtol=1e-11, pc_reuse=100)

    def run(g, p=cfg.params):
        prob.set_params(p)
        prob.set_beta_field(torch.tensor(g, device="cuda"))
        u = torch.tensor(cfg.u0, device="cuda")
        return sk.forward_record(prob, pc, u, steps, cfg.dt, region, 40, ckpt_every=10, **kw)

    try:
        truth = run(si.bump_field(cfg.xy, seed=7)).cpu().numpy()
        g0 = np.ones(cfg.n)
        c = run(g0)
        gg, gnu, st = sk.adjoint(prob, pc, 2 * (c - torch.tensor(truth, device="cuda")), rtol=1e-10)
        gg = gg.cpu().numpy()
        assert st["recomputed_steps"] == 50

        def J(g, p=cfg.params):
            return float(((run(g, p).cpu().numpy() - truth) ** 2).sum())

        h = 1e-6
        for seed in range(100, 120):
            d = si.bump_field(cfg.xy, seed=seed, amp=1.0) - 1.0
            d /= np.abs(d).max()
            fd = (J(g0 + h * d) - J(g0 - h * d)) / (2 * h)
            assert fd == pytest.approx(gg @ d, rel=1e-5), (seed, fd, gg @ d)
        for k in range(5):
            if cfg.params.nu[k] == 0.0:
                continue
            hk = 1e-4 * cfg.params.nu[k]
            nup, num = list(cfg.params.nu), list(cfg.params.nu)
            nup[k] += hk
            num[k] -= hk
            fd = (J(g0, si.Params(**{**cfg.params.__dict__, "nu": tuple(nup)}))
                  - J(g0, si.Params(**{**cfg.params.__dict__, "nu": tuple(num)}))) / (2 * hk)
            assert fd == pytest.approx(gnu[k], rel=1e-5, abs=1e-9 * np.abs(gnu).max()), (k, fd, gnu[k])
    finally:
        prob.set_params(cfg.params)
