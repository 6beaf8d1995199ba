"""Batches: uneven instances with their own rates stepped together equal
the same instances stepped alone (bitwise), and match the oracle."""
import numpy as np
import pytest

import seird_inputs as si
from oracle import fem, newton

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402


def _instances():
    out = []
    xy, tri = si.square_mesh(16)
    p = si.params_square()
    out.append((xy, tri, p, si.square_block_partition(16, 16, 2, 2), 4,
                si.gaussian_bump_state(xy, 1, peak=0.02, width=0.1)))
    c = si.config_realistic(n_base=60, n_ref=2, n_sub=6, seed=11)
    q = si.params_ontario()
    q = si.Params(**{**q.__dict__, "beta_I": 0.012, "beta_E": 0.009,
                     "nu": tuple(np.array(q.nu) * 1.2)})
    out.append((c.xy, c.tri, q, c.part, 6, c.u0))
    xy, tri = si.square_mesh(24)
    r = si.Params(**{**p.__dict__, "beta_I": 0.6, "beta_E": 0.9,
                     "nu": (2e-3, 1e-3, 5e-4, 1.5e-3, 0.0)})
    out.append((xy, tri, r, si.square_block_partition(24, 24, 3, 2), 6,
                si.gaussian_bump_state(xy, 2, peak=0.05, width=0.15)))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_solo_runs_bitwise(prec):
    inst = _instances()
    dt, steps = 0.2, 3
    b = sk.Batch([(x[0], x[1], x[2], x[3], x[4]) for x in inst], overlap=1, factor_prec=prec)
    u = torch.tensor(np.concatenate([x[5] for x in inst]), device="cuda")
    per = []
    for _ in range(steps):
        per.append(b.step(u, dt, tol=1e-10))
    ub = u.cpu().numpy()
    off = b.node_offsets
    for k, x in enumerate(inst):
        prob = sk.Problem(x[0], x[1], x[2])
        pc = sk.Precond(prob, x[3], x[4], 1, factor_prec=prec)
        us = torch.tensor(x[5], device="cuda")
        for n in range(steps):
            st = sk.step(prob, pc, us, dt, tol=1e-10)
            assert st["gmres_its"] == per[n][k]["gmres_its"], (k, n)
        assert np.array_equal(us.cpu().numpy(), ub[off[k]:off[k + 1]]), k


def test_batch_matches_oracle():
    inst = _instances()
    dt = 0.2
    b = sk.Batch([(x[0], x[1], x[2], x[3], x[4]) for x in inst], overlap=2)
    u = torch.tensor(np.concatenate([x[5] for x in inst]), device="cuda")
    b.step(u, dt, tol=1e-13, rtol=1e-10)
    ub = u.cpu().numpy()
    off = b.node_offsets
    for k, x in enumerate(inst):
        geo = fem.Geometry(x[0], x[1])
        uo, _ = newton.newton_step(x[5], dt, geo, x[2], tol=1e-14)
        err = np.linalg.norm(ub[off[k]:off[k + 1]] - uo) / np.linalg.norm(uo)
        assert err < 1e-10, (k, err)


def test_generated_ensemble_equals_solo_runs_and_solves_the_oracle_residual():
    bc = si.config_batch(n_inst=5, n_min=3000, n_max=12000, nodes_per_sub=400, n_ref=1)
    inst = bc.instances
    b = sk.Batch([(c.xy, c.tri, c.params, c.part, c.n_sub) for c in inst],
                 overlap=bc.overlap, factor_prec=1)
    u = torch.tensor(np.concatenate([c.u0 for c in inst]), device="cuda")
    per = b.step(u, bc.dt, tol=1e-10)
    ub = u.cpu().numpy()
    off = b.node_offsets
    for k, c in enumerate(inst):
        prob = sk.Problem(c.xy, c.tri, c.params)
        pc = sk.Precond(prob, c.part, c.n_sub, c.overlap, factor_prec=1)
        us = torch.tensor(c.u0, device="cuda")
        st = sk.step(prob, pc, us, c.dt, tol=1e-10)
        assert st["gmres_its"] == per[k]["gmres_its"], k
        uk = ub[off[k]:off[k + 1]]
        assert np.array_equal(us.cpu().numpy(), uk), k
        geo = fem.Geometry(c.xy, c.tri)
        Fo = fem.residual(uk, c.u0, c.dt, geo, c.params)
        scale = np.linalg.norm(geo.mass[:, None] * c.u0)
        assert np.linalg.norm(Fo) <= 1.01e-10 * scale, k
