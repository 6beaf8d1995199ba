"""The precision workload's required output: each field's error at step 30
against the oracle, for float64, float32 and bfloat16 subdomain factors.
The oracle's state is the stored over-converged step-30 state of the
realistic recipe's nested instance (32,217 nodes, 161,085 unknowns: the
full mesh's recipe and refinement depth with 32x fewer nodes), written by
tests/golden/make_oracle_states.py (oracle Newton with direct solves,
scaled residual 1e-13 every step)."""
import os

import numpy as np
import pytest

import seird_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_polygon32217_r30.npz")


def field_errors(u, ref):
    out = []
    for c in range(5):
        d = u[:, c] - ref[:, c]
        out.append((np.linalg.norm(d) / np.linalg.norm(ref[:, c]), np.abs(d).max() / np.abs(ref[:, c]).max()))
    return out


@pytest.fixture(scope="module")
def nested():
    ref = np.load(REF)
    cfg = si.config_realistic(n_base=int(ref["n_base"]), n_ref=int(ref["n_ref"]), n_sub=32)
    assert cfg.n == int(ref["n_nodes"])
    return cfg, ref


def _run(cfg, prec, steps, **kw):
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, factor_prec=prec,
                    coarse=(cfg.coarse_parents, cfg.coarse_n))
    u = torch.tensor(cfg.u0, device="cuda")
    first = None
    for k in range(steps):
        sk.step(prob, pc, u, cfg.dt, **kw)
        if k == 0:
            first = u.cpu().numpy()
    torch.cuda.synchronize()
    return first, u.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_step30_fields_match_oracle_at_tight_tolerance(nested, prec):
    """Newton to 1e-13, GMRES rtol 1e-10: every field within 1e-8 of the
    oracle's, normwise and in the max norm, whatever the factor precision
    (the root does not depend on it)."""
    cfg, ref = nested
    u1, u30 = _run(cfg, prec, 30, tol=1e-13, rtol=1e-10, pc_reuse=100)
    for c, (l2, linf) in enumerate(field_errors(u1, ref["u1"])):
        assert l2 <= 1e-8 and linf <= 1e-8, ("step 1", c, l2, linf)
    errs = field_errors(u30, ref["u30"])
    print("tight step-30 field errors (l2, max):", [(f"{a:.1e}", f"{b:.1e}") for a, b in errs], flush=True)
    for c, (l2, linf) in enumerate(errs):
        assert l2 <= 1e-8 and linf <= 1e-8, (c, l2, linf)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_step30_fields_at_workload_tolerance(nested, prec):
    """The workload's tolerances (Newton scaled residual 1e-10, GMRES rtol
    1e-5): the step-30 error of every field stays below 1e-6 normwise, the
    bound that a scaled residual of 1e-10 per step allows for the smallest
    field (E, about 1e-4 of S) over 30 steps."""
    cfg, ref = nested
    _, u30 = _run(cfg, prec, 30, tol=cfg.newton_tol, rtol=cfg.gmres_rtol, pc_reuse=100)
    errs = field_errors(u30, ref["u30"])
    print("workload-tolerance step-30 field errors (l2, max):", [(f"{a:.1e}", f"{b:.1e}") for a, b in errs],
          flush=True)
    for c, (l2, linf) in enumerate(errs):
        assert l2 <= 1e-6 and linf <= 1e-6, (c, l2, linf)
