"""Launch-shape choices: the subdomain-solve workgroup sizes give the same
results up to the rounding of a different summation split, and the autotuner reports valid candidates whose best
one builds a preconditioner that solves the oracle's problem."""
import numpy as np
import pytest

import seird_inputs as si
from oracle import fem, newton

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2208_01839_amd as sk  # noqa: E402


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("two_level", [False, True])
def test_solve_widths_agree_to_rounding(prec, two_level):
    cfg = si.config_nested_square(n_base=8, n_ref=2, n_sub=16)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    coarse = (cfg.coarse_parents, cfg.coarse_n) if two_level else None
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, 2, factor_prec=prec, coarse=coarse)
    vals = prob.jacobian(torch.tensor(cfg.u0, device="cuda"), 1.0)
    pc.setup(vals)
    r = torch.tensor(np.random.default_rng(2).standard_normal(prob.N), device="cuda")
    out = {}
    for th in (256, 128, 512, 1024):
        pc.set_solve_threads(th)
        out[th] = (pc.apply(r).cpu().numpy(), pc.apply(r, transpose=True).cpu().numpy())
    for th in (128, 512, 1024):
        for k in (0, 1):  # apply and transposed apply
            a, b = out[th][k], out[256][k]
            assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b), (th, k)
    # repeated applications at one width are bitwise reproducible
    pc.set_solve_threads(512)
    assert np.array_equal(pc.apply(r).cpu().numpy(), out[512][0])


def test_solve_width_rejected_for_tile16():
    cfg = si.config_small()
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, 1, tile=16)
    with pytest.raises(sk.SeirdError):
        pc.set_solve_threads(512)
    with pytest.raises(sk.SeirdError):
        pc.set_solve_threads(300)


def test_autotune_picks_a_valid_fastest_candidate():
    cfg = si.config_nested_square(n_base=8, n_ref=2, n_sub=16)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    coarse = (cfg.coarse_parents, cfg.coarse_n)
    u0 = si.gaussian_bump_state(cfg.xy, 4, peak=0.05, width=0.2)
    vals = prob.jacobian(torch.tensor(u0, device="cuda"), 1.0)
    rep = sk.autotune(prob, cfg.part, cfg.n_sub, 1, vals, coarse=coarse, applies_per_setup=10, reps=3)
    ok = [c for c in rep["candidates"] if c["status"] == 0]
    assert {(c["tile"], c["solve_threads"]) for c in rep["candidates"]} == {(32, 256), (32, 128), (32, 512), (32, 1024),
                                                                           (16, 256)}
    assert ok and all(c["apply_ms"] > 0 and c["setup_ms"] > 0 for c in ok)
    best = min(ok, key=lambda c: c["score_ms"])
    assert (rep["tile"], rep["solve_threads"]) == (best["tile"], best["solve_threads"])
    for c in ok:
        assert abs(c["score_ms"] - (c["setup_ms"] / 10 + c["apply_ms"])) < 1e-9 * c["score_ms"]
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, 1, tile=rep["tile"], coarse=coarse,
                    solve_threads=rep["solve_threads"])
    u = torch.tensor(u0, device="cuda")
    sk.step(prob, pc, u, 1.0, tol=1e-13, rtol=1e-10)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    uo, _ = newton.newton_step(u0, 1.0, geo, cfg.params, tol=1e-14)
    assert np.linalg.norm(u.cpu().numpy() - uo) <= 1e-10 * np.linalg.norm(uo)


def test_autotune_fails_cleanly_when_no_candidate_is_admitted():
    # one subdomain of a 128x128 square: its band (about 650 scalars) is too
    # wide for both tile sizes
    xy, tri = si.square_mesh(128)
    prob = sk.Problem(xy, tri, si.params_square())
    u0 = si.gaussian_bump_state(xy, 0)
    vals = prob.jacobian(torch.tensor(u0, device="cuda"), 0.1)
    with pytest.raises(sk.SeirdError) as e:
        sk.autotune(prob, np.zeros(len(xy), dtype=np.int32), 1, 0, vals, reps=1)
    assert e.value.code == -1


@pytest.mark.parametrize("n_base,n_sub", [(8, 16), (24, 64)])
def test_coarse_inverse_agrees_with_band_sweeps(n_base, n_sub):
    cfg = si.config_nested_square(n_base=n_base, n_ref=2, n_sub=n_sub)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, 2, coarse=(cfg.coarse_parents, cfg.coarse_n))
    u0 = si.gaussian_bump_state(cfg.xy, 4, peak=0.05, width=0.2)
    vals = prob.jacobian(torch.tensor(u0, device="cuda"), 1.0)
    pc.setup(vals)
    r = torch.tensor(np.random.default_rng(5).standard_normal(prob.N), device="cuda")
    out = {}
    for solver in (1, 0):
        pc.set_coarse_solver(solver)
        out[solver] = (pc.apply(r).cpu().numpy(), pc.apply(r, transpose=True).cpu().numpy())
    for k in (0, 1):
        a, b = out[1][k], out[0][k]
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b), k
    with pytest.raises(sk.SeirdError):
        pc.set_coarse_solver(2)


@pytest.mark.gpu
@pytest.mark.parametrize("block", [0, 33, 16, 8])
def test_coarse_block_sweep_agrees_with_band_sweeps(block):
    """Coarse solve by the block sweep over inverted diagonal super-blocks of
    `block` tile rows (0: the full inverses) against the band sweeps over the
    factors, plain and transposed; on this coarse grid (98 tile rows) the
    smaller blocks give 3 to 13 block steps per direction."""
    cfg = si.config_nested_square(n_base=24, n_ref=2, n_sub=64)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, 2, coarse=(cfg.coarse_parents, cfg.coarse_n))
    pc.set_coarse_block(block)
    u0 = si.gaussian_bump_state(cfg.xy, 4, peak=0.05, width=0.2)
    vals = prob.jacobian(torch.tensor(u0, device="cuda"), 1.0)
    pc.setup(vals)
    r = torch.tensor(np.random.default_rng(6).standard_normal(prob.N), device="cuda")
    out = {}
    for solver in (1, 0):
        pc.set_coarse_solver(solver)
        out[solver] = (pc.apply(r).cpu().numpy(), pc.apply(r, transpose=True).cpu().numpy())
    for k in (0, 1):
        a, b = out[1][k], out[0][k]
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b), (block, k)
    with pytest.raises(sk.SeirdError):
        pc.set_coarse_block(1)  # below the coarse band width


def test_autotuner_cache_returns_the_kept_choice(tmp_path, monkeypatch):
    """A second autotune of the same shape comes from the cache (no
    candidate timed) with the same choice; the cache file written through
    SEIRD_TUNE_CACHE holds the key; clearing the cache times again."""
    import seird_inputs as si
    monkeypatch.setenv("SEIRD_TUNE_CACHE", str(tmp_path / "tune.txt"))
    sk.tune_cache_clear()
    cfg = si.config_small(nx=32)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    vals = prob.jacobian(torch.tensor(cfg.u0, device="cuda"), cfg.dt)
    a = sk.autotune(prob, cfg.part, cfg.n_sub, cfg.overlap, vals, reps=2)
    b = sk.autotune(prob, cfg.part, cfg.n_sub, cfg.overlap, vals, reps=2)
    assert not a["from_cache"] and b["from_cache"]
    assert (a["tile"], a["solve_threads"]) == (b["tile"], b["solve_threads"])
    assert len(b["candidates"]) == 0
    sk.tune_cache_clear()
    c = sk.autotune(prob, cfg.part, cfg.n_sub, cfg.overlap, vals, reps=2)
    assert not c["from_cache"] and len(c["candidates"]) > 0
    sk.tune_cache_clear()


def test_batch_autotune_on_the_ensemble():
    import seird_inputs as si
    sk.tune_cache_clear()
    bc = si.config_batch(n_inst=3, n_min=2000, n_max=6000, nodes_per_sub=500)
    b = sk.Batch([(c.xy, c.tri, c.params, c.part, c.n_sub) for c in bc.instances], overlap=bc.overlap)
    u = torch.tensor(np.concatenate([c.u0 for c in bc.instances]), device="cuda")
    b.step(u, bc.dt, tol=1e-10)
    t = b.autotune(reps=2)
    assert t["solve_threads"] in (256, 128, 512, 1024) and len(t["candidates"]) == 4
    assert b.autotune(reps=2)["from_cache"]
    per = b.step(u, bc.dt, tol=1e-10)
    assert all(p["res_hist"][-1] <= 1e-10 for p in per)
    sk.tune_cache_clear()
