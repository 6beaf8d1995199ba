"""GPU Picard-Gauss-Seidel step (the paper's decoupled solver, Appendix A)
against the oracle: its scalar Schwarz preconditioner against the oracle's
one-compartment RAS, the step's result against the oracle's Picard-Gauss-
Seidel fixed point and the coupled Newton root, sweep counts against the
oracle's, through the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp

import seird_inputs as si
from oracle import fem, krylov, newton

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def field_errors(u, ref):
    u, ref = np.asarray(u).reshape(-1, 5), np.asarray(ref).reshape(-1, 5)
    return [np.linalg.norm(u[:, c] - ref[:, c]) / max(np.linalg.norm(ref[:, c]), 1e-300) for c in range(5)]


@pytest.mark.parametrize("tile,overlap", [(16, 1), (32, 2)])
def test_scalar_ras_matches_oracle(tile, overlap):
    cfg = si.config_small(nx=32)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pgs = sk.PicardGS(prob, cfg.part, cfg.n_sub, overlap, tile=tile)
    rp, col = prob.pattern()
    rng = np.random.default_rng(2)
    Nbar = rng.uniform(0.5, 1.5, len(geo.tri))
    A = (sp.diags(geo.mass * rng.uniform(1.0, 2.0, geo.n)) + 0.4 * newton._stiffness(geo, Nbar)).tocsr()
    A.sort_indices()
    diag = A.diagonal()
    rows = np.repeat(np.arange(geo.n), np.diff(rp))
    off = np.asarray(A[rows, col]).ravel()
    pgs.precond.setup_scalar(torch.tensor(diag, device="cuda"), torch.tensor(off, device="cuda"))
    ras = krylov.RAS(A, fem.node_graph(geo), cfg.part, cfg.n_sub, overlap, bs=1)
    r = rng.standard_normal(geo.n)
    z = pgs.precond.apply(torch.tensor(r, device="cuda"))
    torch.cuda.synchronize()
    assert relerr(z.cpu().numpy(), ras.apply(r)) < 1e-11


def _case(vital=False):
    cfg = si.config_small(nx=32)
    kw = {"nu": (0.01, 0.012, 0.005, 0.01, 0.004 if vital else 0.0)}
    if vital:
        kw.update(alpha=0.02, mu=0.01)
    p = si.Params(**{**cfg.params.__dict__, **kw})
    u0 = si.gaussian_bump_state(cfg.xy, 3, peak=0.05, width=0.2)
    return cfg, p, u0


@pytest.mark.parametrize("vital", [False, True])
def test_pgs_step_matches_oracle_fixed_point_and_newton_root(vital):
    cfg, p, u0 = _case(vital)
    dt = 0.3
    geo = fem.Geometry(cfg.xy, cfg.tri)
    g = np.random.default_rng(1).uniform(0.7, 1.3, geo.n) if vital else None
    prob = sk.Problem(cfg.xy, cfg.tri, p)
    if g is not None:
        prob.set_beta_field(torch.tensor(g, device="cuda"))
    pgs = sk.PicardGS(prob, cfg.part, cfg.n_sub, 1)
    u = torch.tensor(u0, device="cuda")
    st = pgs.step(u, dt, tol=1e-13, rtol=1e-12)
    torch.cuda.synchronize()
    ug = u.cpu().numpy()
    uo, info = newton.picard_gs_step(u0, dt, geo, p, g, tol=1e-13)
    un, _ = newton.newton_step(u0, dt, geo, p, g, tol=1e-13)
    assert max(field_errors(ug, uo)) <= 1e-8
    assert max(field_errors(ug, un)) <= 1e-8
    assert abs(st["sweeps"] - info["its"]) <= 1
    assert st["res_scaled"] <= 1e-10
    assert st["eps_hist"][-1] <= 1e-13
    # the solves: every diffusing compartment ran GMRES, D only if it diffuses
    assert all(st["gmres_its"][c] > 0 for c in range(4))
    assert (st["gmres_its"][4] > 0) == vital


def test_pgs_and_newton_steps_agree_on_the_gpu():
    """Ten steps of the small case by both GPU solvers at the workload
    tolerances reach the same states (the root does not depend on the
    iteration)."""
    cfg = si.config_small()
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pgs = sk.PicardGS(prob, cfg.part, cfg.n_sub, cfg.overlap)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap)
    ua = torch.tensor(cfg.u0, device="cuda")
    ub = ua.clone()
    for _ in range(cfg.steps):
        pgs.step(ua, cfg.dt, tol=1e-12, rtol=1e-10)
        sk.step(prob, pc, ub, cfg.dt, tol=1e-12, rtol=1e-10)
    torch.cuda.synchronize()
    assert max(field_errors(ua.cpu().numpy(), ub.cpu().numpy())) <= 1e-8


def test_pgs_reports_non_convergence():
    cfg, p, u0 = _case()
    prob = sk.Problem(cfg.xy, cfg.tri, p)
    pgs = sk.PicardGS(prob, cfg.part, cfg.n_sub, 1)
    u = torch.tensor(u0, device="cuda")
    with pytest.raises(sk.SeirdError) as e:
        pgs.step(u, 0.3, tol=1e-14, max_sweeps=2)
    assert e.value.code == -7


def test_lagged_preconditioners_reach_the_same_fixed_point():
    """With each compartment's preconditioner set up at the first sweep only
    (pc_lag) the step reaches the same fixed point with one setup per
    diffusing compartment, on two steps in a row (the second sets up anew)."""
    cfg, p, u0 = _case()
    geo = fem.Geometry(cfg.xy, cfg.tri)
    prob = sk.Problem(cfg.xy, cfg.tri, p)
    pgs = sk.PicardGS(prob, cfg.part, cfg.n_sub, 1)
    ua = torch.tensor(u0, device="cuda")
    ub = ua.clone()
    uo = u0.copy()
    for _ in range(2):
        sa = pgs.step(ua, 0.3, tol=1e-13, rtol=1e-12)
        sb = pgs.step(ub, 0.3, tol=1e-13, rtol=1e-12, pc_lag=True)
        uo, _ = newton.picard_gs_step(uo, 0.3, geo, p, None, tol=1e-13)
        assert sb["pc_setups"] == 4 and sa["pc_setups"] == 4 * sa["sweeps"]
        assert abs(sb["sweeps"] - sa["sweeps"]) <= 1
        assert sb["res_scaled"] <= 1e-10
    torch.cuda.synchronize()
    assert max(field_errors(ub.cpu().numpy(), uo)) <= 1e-8
    assert max(field_errors(ub.cpu().numpy(), ua.cpu().numpy())) <= 1e-9
