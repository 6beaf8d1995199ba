"""GPU discrete adjoint against the oracle's adjoint and against central
finite differences of GPU forward runs (h = 1e-6, random directions,
1e-5 relative)."""
import numpy as np
import pytest

import seird_inputs as si
from oracle import adjoint as oadj
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402

TIGHT = dict(tol=1e-13, rtol=1e-11)
ADJ = dict(rtol=1e-11)


def _case(nested=False):
    if nested:
        cfg = si.config_nested_square(n_base=4, n_ref=2, n_sub=4)
        xy, tri = cfg.xy, cfg.tri
        part, n_sub, coarse = cfg.part, cfg.n_sub, (cfg.coarse_parents, cfg.coarse_n)
    else:
        xy, tri = si.square_mesh(12)
        part, n_sub, coarse = si.square_block_partition(12, 12, 2, 2), 4, None
    p = si.Params(**{**si.params_square().__dict__, "nu": (0.02, 0.015, 0.01, 0.02, 0.005)})
    u0 = si.gaussian_bump_state(xy, 3, peak=0.05, width=0.25)
    g = np.random.default_rng(0).uniform(0.8, 1.2, len(xy))
    region = (xy[:, 0] > 0.5).astype(np.int32) + 2 * (xy[:, 1] > 0.5).astype(np.int32)
    region[::7] = -1
    return xy, tri, p, u0, g, region, part, n_sub, coarse


def _gpu_forward(prob, pc, p, u0, g, region, steps, dt, ckpt=3):
    prob.set_params(p)
    prob.set_beta_field(torch.tensor(g, device="cuda"))
    u = torch.tensor(u0, device="cuda")
    c = sk.forward_record(prob, pc, u, steps, dt, region, 4, ckpt_every=ckpt, **TIGHT)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("nested", [False, True])
def test_adjoint_matches_oracle_adjoint(nested):
    xy, tri, p, u0, g, region, part, n_sub, coarse = _case(nested)
    steps, dt = 7, 0.5
    prob = sk.Problem(xy, tri, p)
    pc = sk.Precond(prob, part, n_sub, 1, coarse=coarse)
    c = _gpu_forward(prob, pc, p, u0, g, region, steps, dt)
    geo = fem.Geometry(xy, tri)
    states, co = oadj.forward(u0, steps, dt, geo, p, g, region, 4, tol=1e-14)
    assert np.abs(c - co).max() <= 1e-9 * np.abs(co).max()
    target = co * 0.9 + 1e-4
    gc = 2 * (co - target)
    gg, gnu, st = sk.adjoint(prob, pc, torch.tensor(gc, device="cuda"), **ADJ)
    ogg, ognu = oadj.adjoint_gradient(states, dt, geo, p, g, region, 4, gc)
    gg = gg.cpu().numpy()
    assert np.linalg.norm(gg - ogg) <= 1e-7 * np.linalg.norm(ogg)
    assert np.abs(gnu - ognu).max() <= 1e-7 * np.abs(ognu).max()
    assert st["recomputed_steps"] == 6  # segments of 3: steps 1-6 recomputed, 7 kept


def test_adjoint_matches_finite_differences():
    xy, tri, p, u0, g, region, part, n_sub, coarse = _case()
    steps, dt = 5, 0.5
    prob = sk.Problem(xy, tri, p)
    pc = sk.Precond(prob, part, n_sub, 1)
    c = _gpu_forward(prob, pc, p, u0, g, region, steps, dt)
    target = c * 0.9 + 1e-4

    def J(gv, pv):
        cc = _gpu_forward(prob, pc, pv, u0, gv, region, steps, dt)
        return float(((cc - target) ** 2).sum())

    _gpu_forward(prob, pc, p, u0, g, region, steps, dt)
    gg, gnu, _ = sk.adjoint(prob, pc, torch.tensor(2 * (c - target), device="cuda"), **ADJ)
    gg = gg.cpu().numpy()
    rng = np.random.default_rng(9)
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(len(xy))
        d /= np.abs(d).max()
        fd = (J(g + h * d, p) - J(g - h * d, p)) / (2 * h)
        assert fd == pytest.approx(gg @ d, rel=1e-5)
    for cidx in range(5):
        hc = 1e-4 * p.nu[cidx]
        nu_p, nu_m = np.array(p.nu), np.array(p.nu)
        nu_p[cidx] += hc
        nu_m[cidx] -= hc
        fd = (J(g, si.Params(**{**p.__dict__, "nu": tuple(nu_p)}))
              - J(g, si.Params(**{**p.__dict__, "nu": tuple(nu_m)}))) / (2 * hc)
        assert fd == pytest.approx(gnu[cidx], rel=1e-5, abs=1e-9 * np.abs(gnu).max())


def test_autograd_function_backward():
    xy, tri, p, u0, g, region, part, n_sub, coarse = _case()
    steps, dt = 4, 0.5
    prob = sk.Problem(xy, tri, p)
    pc = sk.Precond(prob, part, n_sub, 1)
    gt = torch.tensor(g, device="cuda", requires_grad=True)
    nut = torch.tensor(p.nu, dtype=torch.float64, device="cuda", requires_grad=True)
    opts = dict(base_params=p, ckpt_every=2, tol=1e-13, krylov=dict(rtol=1e-11),
                adjoint_krylov=dict(rtol=1e-11))
    counts = sk.SEIRDRun.apply(gt, nut, prob, pc, torch.tensor(u0, device="cuda"), steps, dt,
                               region, 4, opts)
    target = counts.detach() * 1.1
    loss = ((counts - target) ** 2).sum()
    loss.backward()
    geo = fem.Geometry(xy, tri)
    states, co = oadj.forward(u0, steps, dt, geo, p, g, region, 4, tol=1e-14)
    ogg, ognu = oadj.adjoint_gradient(states, dt, geo, p, g, region, 4,
                                      2 * (co - target.cpu().numpy()))
    assert np.linalg.norm(gt.grad.cpu().numpy() - ogg) <= 1e-7 * np.linalg.norm(ogg)
    assert np.abs(nut.grad.cpu().numpy() - ognu).max() <= 1e-7 * np.abs(ognu).max()


def test_kept_setups_match_the_oracle_adjoint():
    """pc_keep_steps: a setup kept across the steps of a checkpoint segment,
    forward and in the transposed solves, reaches the oracle's gradient; the
    reverse sweep makes fewer setups than it has steps."""
    xy, tri, p, u0, g, region, part, n_sub, coarse = _case(True)
    steps, dt = 7, 0.5
    prob = sk.Problem(xy, tri, p)
    pc = sk.Precond(prob, part, n_sub, 1, coarse=coarse)
    prob.set_params(p)
    prob.set_beta_field(torch.tensor(g, device="cuda"))
    u = torch.tensor(u0, device="cuda")
    c = sk.forward_record(prob, pc, u, steps, dt, region, 4, ckpt_every=3, pc_keep_steps=2,
                          **TIGHT).cpu().numpy()
    geo = fem.Geometry(xy, tri)
    states, co = oadj.forward(u0, steps, dt, geo, p, g, region, 4, tol=1e-14)
    assert np.abs(c - co).max() <= 1e-9 * np.abs(co).max()
    gc = 2 * (co - (co * 0.9 + 1e-4))
    gg, gnu, st = sk.adjoint(prob, pc, torch.tensor(gc, device="cuda"), **ADJ)
    ogg, ognu = oadj.adjoint_gradient(states, dt, geo, p, g, region, 4, gc)
    assert np.linalg.norm(gg.cpu().numpy() - ogg) <= 1e-7 * np.linalg.norm(ogg)
    assert np.abs(gnu - ognu).max() <= 1e-7 * np.abs(ognu).max()
    assert st["recomputed_steps"] == 6
    assert 3 <= st["setups"] < steps  # one per segment at least; segments of 3, 3, 1
    # without keeping, one setup per reverse step
    u = torch.tensor(u0, device="cuda")
    sk.forward_record(prob, pc, u, steps, dt, region, 4, ckpt_every=3, **TIGHT)
    _, _, st0 = sk.adjoint(prob, pc, torch.tensor(gc, device="cuda"), **ADJ)
    assert st0["setups"] == steps


def test_one_segment_record_keeps_every_state_and_gives_the_same_gradient():
    """ckpt_every >= n_steps: every state of the run stays in device memory,
    the reverse sweep recomputes nothing, and the gradient is the one of a
    checkpointed record of the same run."""
    xy, tri, p, u0, g, region, part, n_sub, coarse = _case(True)
    steps, dt = 7, 0.5
    prob = sk.Problem(xy, tri, p)
    pc = sk.Precond(prob, part, n_sub, 1, coarse=coarse)
    out = {}
    for ckpt in (3, steps):
        c = _gpu_forward(prob, pc, p, u0, g, region, steps, dt, ckpt=ckpt)
        gc = 2 * (c - (c * 0.9 + 1e-4))
        gg, gnu, st = sk.adjoint(prob, pc, torch.tensor(gc, device="cuda"), **ADJ)
        out[ckpt] = (c, gg.cpu().numpy(), gnu, st)
    assert out[steps][3]["recomputed_steps"] == 0
    assert out[3][3]["recomputed_steps"] == 6
    assert np.array_equal(out[3][0], out[steps][0])  # the same forward run
    assert np.linalg.norm(out[3][1] - out[steps][1]) <= 1e-12 * np.linalg.norm(out[3][1])
    assert np.abs(out[3][2] - out[steps][2]).max() <= 1e-12 * np.abs(out[3][2]).max()
