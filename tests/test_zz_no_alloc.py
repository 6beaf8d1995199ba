"""GPU test of seird_gmres_noalloc (the allocation-free GMRES whose scratch
is the library's fixed per-GPU array) against seird_gmres, through the C
ABI: two calls in a row, the second on a smaller problem, each bitwise equal
to the allocating entry point's result, with no change of the device's free
memory across the allocation-free calls."""
import numpy as np
import pytest

import seird_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402


def _system(nx, two_level=False, seed=0):
    if two_level:
        cfg = si.config_nested_square(n_base=4, n_ref=2, n_sub=4)
        coarse = (cfg.coarse_parents, cfg.coarse_n)
    else:
        cfg = si.config_small(nx=nx)
        coarse = None
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, coarse=coarse)
    u = torch.tensor(cfg.u0, device="cuda")
    vals = prob.jacobian(u, 2.0)
    pc.setup(vals)
    b = torch.tensor(np.random.default_rng(seed).standard_normal(prob.N), device="cuda")
    return prob, pc, vals, b


def test_noalloc_gmres_equals_gmres_on_two_calls():
    cases = [(64, False, 0), (16, True, 1)]   # 21,125 unknowns, then 1,445
    systems = [_system(*c) for c in cases]
    for transpose in (False, True):
        refs = []
        for prob, pc, vals, b in systems:
            x, st = sk.gmres(prob, pc, vals, b, transpose=transpose, rtol=1e-10)
            torch.cuda.synchronize()
            refs.append((x.clone(), st))
        xs = [torch.full_like(b, float("nan")) for _, _, _, b in systems]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        sts = []
        for (prob, pc, vals, b), x in zip(systems, xs):
            sts.append(sk.gmres_noalloc(prob, pc, vals, b, x, transpose=transpose, rtol=1e-10))
            torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        for (prob, pc, vals, b), x, st, (xr, sr) in zip(systems, xs, sts, refs):
            assert st["reason"] == sr["reason"] and st["its"] == sr["its"]
            assert torch.equal(x, xr)
            assert torch.linalg.norm(prob.spmv(vals, x, transpose=transpose) - b) <= 1e-9 * torch.linalg.norm(b)


def test_noalloc_gmres_rejects_a_basis_above_the_scratch():
    prob, pc, vals, b = _system(64)
    N = prob.N
    # restart 30 on 21,125 unknowns fits; a problem whose basis exceeds
    # SEIRD_STATIC_SCRATCH_BYTES is rejected before any launch
    big = si.config_small(nx=200)  # 201^2 nodes -> 202,005 unknowns
    pb = sk.Problem(big.xy, big.tri, big.params)
    vb = pb.jacobian(torch.tensor(big.u0, device="cuda"), 0.1)
    bb = torch.ones(pb.N, dtype=torch.float64, device="cuda")
    xb = torch.zeros_like(bb)
    assert (2 * 30 + 1) * pb.N * 8 > sk.STATIC_SCRATCH_BYTES
    with pytest.raises(sk.SeirdError) as e:
        sk.gmres_noalloc(pb, None, vb, bb, xb, restart=30)
    assert e.value.code == -1
    # the same problem with a short restart fits
    st = sk.gmres_noalloc(pb, None, vb, bb, xb, restart=4, max_it=8)
    xr, sr = sk.gmres(pb, None, vb, bb, restart=4, max_it=8)
    torch.cuda.synchronize()
    assert st["its"] == sr["its"] and torch.equal(xb, xr)
    assert N > 0
