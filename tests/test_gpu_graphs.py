"""Arnoldi steps replayed from captured HIP graphs give exactly the results
of direct launches: one- and two-level steps, restarts, batches and the
transposed (adjoint) solves.  Every graph is replayed many times, with the
program's own eager work and synchronisations in between."""
import numpy as np
import pytest

import seird_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402


def _run_steps(prob, pc, u0, dt, steps, graphs, **kw):
    u = torch.tensor(u0, device="cuda")
    its = []
    for _ in range(steps):
        st = sk.step(prob, pc, u, dt, graphs=graphs, **kw)
        its.append(st["gmres_its"])
    return u.cpu().numpy(), its


@pytest.mark.parametrize("two_level", [False, True])
def test_graph_steps_equal_direct_launches(two_level):
    cfg = si.config_nested_square(n_base=8, n_ref=2, n_sub=16)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    coarse = (cfg.coarse_parents, cfg.coarse_n) if two_level else None
    u0 = si.gaussian_bump_state(cfg.xy, 4, peak=0.05, width=0.2)
    kw = dict(tol=1e-12, rtol=1e-8)
    pc0 = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse)
    u_a, its_a = _run_steps(prob, pc0, u0, 1.0, 4, 0, **kw)
    pc1 = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse)
    u_b, its_b = _run_steps(prob, pc1, u0, 1.0, 4, 1, **kw)   # captures
    u_c, its_c = _run_steps(prob, pc1, u0, 1.0, 4, 1, **kw)   # replays the cache
    assert sum(map(sum, its_a)) > 10
    assert its_a == its_b == its_c
    assert np.array_equal(u_a, u_b) and np.array_equal(u_a, u_c)


def test_graph_restarts_equal_direct_launches():
    cfg = si.config_small()
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    vals = prob.jacobian(torch.tensor(cfg.u0, device="cuda"), 5.0)
    pc.setup(vals)
    b = torch.tensor(np.random.default_rng(1).standard_normal(5 * cfg.n), device="cuda")
    xs = []
    for graphs in (0, 1, 1):
        x, st = sk.gmres(prob, pc, vals, b, restart=4, rtol=1e-10, max_it=200, graphs=graphs)
        xs.append((x.cpu().numpy(), st["its"]))
    assert xs[0][1] > 8  # several restart cycles
    for x, its in xs[1:]:
        assert np.array_equal(x, xs[0][0]) and its == xs[0][1]


def test_graph_batch_and_adjoint_equal_direct_launches():
    bc = si.config_batch(n_inst=3, n_min=2000, n_max=6000, nodes_per_sub=400, n_ref=1)
    inst = [(c.xy, c.tri, c.params, c.part, c.n_sub) for c in bc.instances]
    u0 = np.concatenate([c.u0 for c in bc.instances])
    res = []
    for graphs in (0, 1):
        b = sk.Batch(inst, overlap=2)
        u = torch.tensor(u0, device="cuda")
        per = [b.step(u, 1.0, graphs=graphs) for _ in range(2)]
        res.append((u.cpu().numpy(), [[p["gmres_its"] for p in q] for q in per]))
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]

    c = bc.instances[0]
    prob = sk.Problem(c.xy, c.tri, c.params)
    pc = sk.Precond(prob, c.part, c.n_sub, 2)
    region = si.voronoi_regions(c.xy, 6, seed=8)
    grads = []
    for graphs in (0, 1):
        u = torch.tensor(c.u0, device="cuda")
        counts = sk.forward_record(prob, pc, u, 4, 1.0, region, 6, ckpt_every=2, graphs=graphs)
        gg, gnu, _ = sk.adjoint(prob, pc, counts * 0.1, rtol=1e-9, graphs=graphs)
        grads.append((counts.cpu().numpy(), gg.cpu().numpy(), gnu))
    for a, b2 in zip(grads[0], grads[1]):
        assert np.array_equal(a, b2)
