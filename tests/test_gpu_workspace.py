"""The caller-owned-workspace boundary (seird_mesh_create,
seird_workspace_bytes, seird_create_in_workspace) and the scalar-CSR export
of the Jacobian (seird_csr, seird_csr_values), through the C ABI: results
equal to the library-owned path, no device allocation by the library, and
the CSR values against the node-block storage and the oracle's Jacobian."""
import numpy as np
import pytest
import scipy.sparse as sp

import seird_inputs as si
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402

TIGHT = dict(tol=1e-12, rtol=1e-10)


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _record_and_adjoint(prob, pc, u0, region, steps=5, dt=0.5):
    u = torch.tensor(u0, device="cuda")
    c = sk.forward_record(prob, pc, u, steps, dt, region, 4, ckpt_every=2, **TIGHT)
    g, gnu, _ = sk.adjoint(prob, pc, 2 * c, rtol=1e-11)
    torch.cuda.synchronize()
    return c.clone(), g.clone(), gnu, u.clone()


def test_one_level_problem_in_workspace_allocates_nothing():
    cfg = si.config_small(nx=32)
    region = (cfg.xy[:, 0] > 0.5).astype(np.int32) + 2 * (cfg.xy[:, 1] > 0.5).astype(np.int32)
    # the library-owned path first: reference results, and the torch
    # allocations of the binding (counts, gradients) land in torch's cache
    ref_prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    ref_pc = sk.Precond(ref_prob, cfg.part, cfg.n_sub, cfg.overlap)
    u_ref = torch.tensor(cfg.u0, device="cuda")
    sk.step(ref_prob, ref_pc, u_ref, cfg.dt, **TIGHT)
    ref_rec = _record_and_adjoint(ref_prob, ref_pc, cfg.u0, region)
    mesh = sk.Mesh(cfg.xy, cfg.tri)
    # n_steps 5, checkpoints every 2: 3 + 2 + 4 tape states
    ws_kw = dict(restart_max=30, tape_states=9, n_regions_max=4)
    nbytes = sk.workspace_bytes(mesh, cfg.part, cfg.n_sub, cfg.overlap, **ws_kw)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    u = torch.tensor(cfg.u0, device="cuda")
    free0 = _free()
    allocs0 = sk.device_allocations()
    prob, pc = sk.create_in_workspace(mesh, cfg.params, ws, cfg.part, cfg.n_sub, cfg.overlap, **ws_kw)
    st = sk.step(prob, pc, u, cfg.dt, **TIGHT)
    rec = _record_and_adjoint(prob, pc, cfg.u0, region)
    assert sk.device_allocations() == allocs0
    assert _free() == free0
    assert st["reason"] == 0
    assert torch.equal(u, u_ref)
    for a, b in zip(rec, ref_rec):
        if isinstance(a, np.ndarray):
            assert np.array_equal(a, b)
        else:
            assert torch.equal(a, b)
    del pc, prob
    torch.cuda.synchronize()


def test_two_level_problem_in_workspace_matches_library_owned():
    cfg = si.config_nested_square(n_base=8, n_ref=2, n_sub=8)
    coarse = (cfg.coarse_parents, cfg.coarse_n)
    ref_prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    ref_pc = sk.Precond(ref_prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse)
    u_ref = torch.tensor(cfg.u0, device="cuda")
    for _ in range(3):
        sk.step(ref_prob, ref_pc, u_ref, 2.0, **TIGHT)
    mesh = sk.Mesh(cfg.xy, cfg.tri)
    nbytes = sk.workspace_bytes(mesh, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse, restart_max=30)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    u = torch.tensor(cfg.u0, device="cuda")
    allocs0 = sk.device_allocations()
    prob, pc = sk.create_in_workspace(mesh, cfg.params, ws, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse,
                                      restart_max=30)
    sk.step(prob, pc, u, 2.0, **TIGHT)
    # no device allocation by the library from creation on; the free-memory
    # check starts after the first step, by which the HIP runtime has set
    # up its own resources for the preconditioner's second stream
    free0 = _free()
    for _ in range(2):
        sk.step(prob, pc, u, 2.0, **TIGHT)
    assert sk.device_allocations() == allocs0
    assert _free() == free0
    assert torch.equal(u, u_ref)


def test_workspace_limits_are_reported():
    cfg = si.config_small(nx=16)
    mesh = sk.Mesh(cfg.xy, cfg.tri)
    nbytes = sk.workspace_bytes(mesh, cfg.part, cfg.n_sub, 1, restart_max=10)
    small = torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(sk.SeirdError) as e:
        sk.create_in_workspace(mesh, cfg.params, small, cfg.part, cfg.n_sub, 1, restart_max=10)
    assert e.value.code == -8
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    prob, pc = sk.create_in_workspace(mesh, cfg.params, ws, cfg.part, cfg.n_sub, 1, restart_max=10)
    u = torch.tensor(cfg.u0, device="cuda")
    with pytest.raises(sk.SeirdError) as e:   # restart above the reservation
        sk.step(prob, pc, u, cfg.dt, restart=30)
    assert e.value.code == -8
    st = sk.step(prob, pc, u, cfg.dt, restart=10)
    assert st["reason"] == 0
    region = np.zeros(cfg.n, np.int32)
    with pytest.raises(sk.SeirdError) as e:   # no tape reserved
        sk.forward_record(prob, pc, u, 2, cfg.dt, region, 1, ckpt_every=1, restart=10)
    assert e.value.code == -8
    with pytest.raises(sk.SeirdError) as e:   # no CSR pattern reserved
        prob.csr()
    assert e.value.code == -8


def test_problem_from_mesh_equals_problem_from_arrays():
    cfg = si.config_small(nx=16)
    a = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    b = sk.Problem.from_mesh(sk.Mesh(cfg.xy, cfg.tri), cfg.params)
    u = torch.tensor(cfg.u0 * 1.1, device="cuda")
    up = torch.tensor(cfg.u0, device="cuda")
    assert torch.equal(a.residual(u, up, 0.1), b.residual(u, up, 0.1))
    assert torch.equal(a.jacobian(u, 0.1), b.jacobian(u, 0.1))


def test_scalar_csr_matches_node_blocks_and_oracle():
    cfg = si.config_small(nx=16)
    p = si.Params(**{**cfg.params.__dict__, "nu": (1e-3, 2e-3, 5e-4, 1e-3, 3e-4)})
    prob = sk.Problem(cfg.xy, cfg.tri, p)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    rng = np.random.default_rng(3)
    u = cfg.u0 * rng.uniform(0.8, 1.2, cfg.u0.shape) + rng.uniform(0, 0.01, cfg.u0.shape)
    ut = torch.tensor(u, device="cuda")
    vals = prob.jacobian(ut, 0.21)
    rp, col = prob.csr()
    cv = prob.csr_values(vals).cpu().numpy()
    N = 5 * cfg.n
    assert len(rp) == N + 1 and rp[-1] == len(col) == 25 * (prob.nslots + cfg.n)
    assert np.all(np.diff(col.astype(np.int64))[np.diff(np.repeat(np.arange(N), np.diff(rp))) == 0] > 0)
    J = sp.csr_matrix((cv, col, rp), shape=(N, N))
    Jo = fem.jacobian(u, 0.21, geo, p)
    D = (J - Jo).tocoo()
    assert np.abs(D.data).max(initial=0) <= 1e-13 * np.abs(Jo.data).max()
    x = rng.standard_normal(N)
    y = prob.spmv(vals, torch.tensor(x, device="cuda")).cpu().numpy()
    assert np.linalg.norm(J @ x - y) <= 1e-13 * np.linalg.norm(y)
