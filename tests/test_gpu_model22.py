"""The 22-compartment model (Appendix C) on the GPU against the oracle's
``model22``: residual, one decoupled Picard-Gauss-Seidel step, several steps
with diffusion, conservation and the zero-diffusion ODE limit, through the
C ABI."""
import dataclasses

import numpy as np
import pytest

import seird_inputs as si
from oracle import fem, model22 as m22

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
def case():
    xy, tri = si.square_mesh(40)
    part = si.square_block_partition(40, 40, 4, 4)
    p = si.Params22(nu=(2e-3, 2e-3, 2e-3, 1e-3, 1e-3, 5e-4, 2e-4, 5e-4, 2e-3, 2e-3))
    u0 = si.state22(xy, 3, peak=0.05, width=0.12)
    mesh = sk.Mesh(xy, tri)
    model = sk.Model22(mesh, p, part, 16, 1)
    return xy, tri, part, p, u0, mesh, model, fem.Geometry(xy, tri)


def test_residual_matches_oracle(case):
    xy, tri, part, p, u0, mesh, model, geo = case
    rng = np.random.default_rng(5)
    u = u0 * rng.uniform(0.8, 1.2, u0.shape) + rng.uniform(0, 1e-3, u0.shape)
    F = H(model.residual(T(u), T(u0), 0.7))
    Fo = m22.residual22(u, u0, 0.7, geo, p)
    assert relerr(F, Fo) < 1e-13
    assert np.abs(F - Fo).max() <= 1e-13 * np.abs(Fo).max()


def test_one_step_matches_the_oracle_sweeps(case):
    xy, tri, part, p, u0, mesh, model, geo = case
    u = T(u0)
    st = model.step(u, 1.0, tol=1e-13, rtol=1e-12)
    uo, hist = m22.picard_gs_step22(u0, 1.0, geo, p, tol=1e-13)
    ug = H(u)
    for c in range(m22.NC22):
        scale = max(np.abs(uo[:, c]).max(), 1e-30)
        assert np.abs(ug[:, c] - uo[:, c]).max() <= 1e-10 * max(scale, 1e-12 * np.abs(uo).max()), m22.NAMES[c]
    assert abs(st["sweeps"] - len(hist)) <= 1, (st["sweeps"], len(hist))
    assert st["res_scaled"] < 1e-11
    assert st["pc_setups"] == 10


def test_steps_conserve_population_and_reuse_constant_preconditioners(case):
    xy, tri, part, p, u0, mesh, model, geo = case
    u = T(u0)
    uo = u0.copy()
    setups = []
    for _ in range(3):
        st = model.step(u, 2.0, tol=1e-12, rtol=1e-10)
        setups.append(st["pc_setups"])
        uo, _ = m22.picard_gs_step22(uo, 2.0, geo, p, tol=1e-13)
    ug = H(u)
    assert relerr(ug, uo) < 1e-9
    tot0 = (geo.mass[:, None] * u0).sum()
    assert abs((geo.mass[:, None] * ug).sum() - tot0) <= 1e-10 * tot0
    assert ug.min() >= -1e-12
    # a new dt sets every diffusing compartment up once; later steps only S and V
    assert setups[0] == 10 and setups[1] == 2 and setups[2] == 2, setups


def test_zero_diffusion_is_the_nodal_ode(case):
    xy, tri, part, p, u0, mesh, model, geo = case
    q = dataclasses.replace(p, nu=(0.0,) * 10)
    model.set_params(q)
    try:
        u = T(u0)
        st = model.step(u, 1.0, tol=1e-14)
        uo, _ = m22.picard_gs_step22(u0, 1.0, geo, q, tol=1e-14)
        assert relerr(H(u), uo) < 1e-12
        assert sum(st["gmres_its"]) == 0 and st["pc_setups"] == 0
    finally:
        model.set_params(p)


def test_errors(case):
    xy, tri, part, p, u0, mesh, model, geo = case
    bad = u0.copy()
    bad[3, 7] = np.nan
    with pytest.raises(sk.SeirdError) as e:
        model.step(T(bad), 1.0)
    assert e.value.code == -4
    with pytest.raises(sk.SeirdError) as e:
        model.step(T(u0), 1.0, tol=1e-30, max_sweeps=2)
    assert e.value.code == -7
    with pytest.raises(sk.SeirdError) as e:
        sk.Model22(mesh, dataclasses.replace(p, gamma_E=-1.0), part, 16, 1)
    assert e.value.code == -1
