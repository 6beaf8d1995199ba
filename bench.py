#!/usr/bin/env python3
"""Benchmark of the SEIRD implicit step on one MI355X.

A "step" is one backward-Euler time step of the realistic workload (seeded
star polygon, ~1.01M P1 nodes = ~5.05M unknowns, Ontario rates, dt = 1 day):
Newton iterations, each with residual and Jacobian assembly, two-grid RAS
setup (1024 subdomains, overlap 2, nested coarse grid 4 refinement levels
coarser, Galerkin coarse matrix) and GMRES(30) to rtol 1e-5, until the
scaled residual is below 1e-10.  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  --prec selects the storage precision of the
subdomain factors of the main leg (0 FP64, 1 FP32, 2 BF16); unless
--no-compare-prec, FP32 and BF16 legs on the same steps follow and are
reported in "mixed".  The ensemble leg ("batch") steps 48 uneven instances
together; the adjoint leg ("adjoint") times one misfit gradient.  The CPU
baseline is the FP64 oracle (numpy/scipy) timed on a bounded sample of the
same workload (a nested mesh of the same kind with 32x fewer nodes, same
subdomain size), scaled to 5M unknowns by the unknown ratio.
"""
import argparse
import json
import os
import sys
import time

PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the subdomain-solve kernel from rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE, copy-calibrated) of the current kernel, by
# (factor precision, tile, solve threads); the table and commands are in
# profiles/traffic_realistic_fp64.md.  Legs without a measurement report null.
MEASURED_SOLVE_TRAFFIC = {(0, 32, 256): (20.926 + 0.177) * 1e9, (0, 32, 512): (20.858 + 0.178) * 1e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(args):
    import seird_inputs as si
    if args.workload == "small":
        cfg = si.config_small()
        coarse = None
    else:
        cfg = si.config_realistic(n_base=args.n_base, n_ref=args.n_ref, n_sub=args.n_sub)
        coarse = (cfg.coarse_parents, cfg.coarse_n)
    return cfg, coarse


def run_steps(sk, torch, cfg, coarse, prec, steps, warmup, tile, pc_reuse=0, threads=256):
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    tune = None
    if tile == "auto":
        # launch shapes chosen by the autotuner on the first Jacobian (untimed)
        vals = prob.jacobian(torch.tensor(cfg.u0, dtype=torch.float64, device="cuda"), cfg.dt)
        tune = sk.autotune(prob, cfg.part, cfg.n_sub, cfg.overlap, vals, factor_prec=prec,
                           coarse=coarse, applies_per_setup=15, reps=3)
        del vals
        tile, threads = tune["tile"], tune["solve_threads"]
        log(f"[bench] prec={prec} autotune: tile {tile}, solve threads {threads}; "
            + ", ".join(f"({c['tile']},{c['solve_threads']}): "
                        + (f"setup {c['setup_ms']:.1f} apply {c['apply_ms']:.2f} ms" if c["status"] == 0
                           else f"status {c['status']}") for c in tune["candidates"]))
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, tile=tile,
                    factor_prec=prec, coarse=coarse, solve_threads=threads)
    pc.enable_timing(True)
    info = pc.info()
    u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
    kw = dict(tol=cfg.newton_tol, max_it=cfg.newton_max_it, restart=cfg.gmres_restart,
              rtol=cfg.gmres_rtol, atol=cfg.gmres_atol, dtol=cfg.gmres_dtol, pc_reuse=pc_reuse)
    for w in range(warmup):
        st = sk.step(prob, pc, u, cfg.dt, **kw)
        log(f"[bench] prec={prec} warmup step {w}: newton={st['newton_its']} gmres={st['gmres_its']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        st = sk.step(prob, pc, u, cfg.dt, **kw)
        stats.append(st)
        log(f"[bench] prec={prec} reuse={pc_reuse} step {k}: newton={st['newton_its']} setups={st['pc_setups']} gmres={st['gmres_its']} "
            f"res={st['res_hist'][-1]:.2e} t(res/jac/setup/gmres)ms="
            f"{st['t_residual_ms']:.1f}/{st['t_jacobian_ms']:.1f}/{st['t_setup_ms']:.1f}/{st['t_gmres_ms']:.1f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return dict(seconds=t1 - t0, stats=stats, info=info, u=u, tile=tile, solve_threads=threads, tune=tune)


def adjoint_bench(sk, torch, args, cfg, coarse):
    """One gradient of the case-count misfit (forward record + reverse
    sweep) with respect to the per-node transmission field and the five
    diffusion coefficients; checkpoints every 10 steps (5 for short runs)."""
    import numpy as np
    import seird_inputs as si
    if args.adjoint_full:
        cfg = si.config_differentiation()
        coarse = (cfg.coarse_parents, cfg.coarse_n)
        steps, every = cfg.steps, 10
    else:
        steps = args.adjoint_steps
        every = 10 if steps >= 20 else 5
    region = si.voronoi_regions(cfg.xy, 40, seed=8)
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    tile, threads = args.tuned.get(0, (32, 256))
    pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, tile=tile, coarse=coarse,
                    solve_threads=threads)
    kw = dict(tol=cfg.newton_tol, pc_reuse=args.pc_reuse, rtol=cfg.gmres_rtol)
    # synthetic truth: the same run with the perturbed transmission field
    g_true = torch.tensor(si.bump_field(cfg.xy, seed=7), device="cuda")
    prob.set_beta_field(g_true)
    u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
    log(f"[bench] adjoint: {cfg.name}, {steps} steps; truth run")
    truth = sk.forward_record(prob, pc, u, steps, cfg.dt, region, 40, ckpt_every=every, **kw)
    log("[bench] adjoint: timed forward record")
    prob.set_beta_field(torch.ones(cfg.n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
    counts = sk.forward_record(prob, pc, u, steps, cfg.dt, region, 40, ckpt_every=every, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[bench] adjoint: forward {t1 - t0:.2f} s; reverse sweep")
    grad_g, grad_nu, st = sk.adjoint(prob, pc, 2 * (counts - truth), rtol=1e-8)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"[bench] adjoint: forward {t1 - t0:.2f} s, reverse {t2 - t1:.2f} s, {st}")
    return {"metric": "adjoint gradients/s", "value": 1.0 / (t2 - t0), "unit": "grads/s",
            "workload": (f"{cfg.name}: {cfg.n} nodes ({5 * cfg.n} unknowns), {steps} daily steps, "
                         f"checkpoint every {every}, 40 Voronoi regions, gradient w.r.t. the per-node "
                         f"transmission field and 5 diffusion coefficients"),
            "forward_s": t1 - t0, "reverse_s": t2 - t1,
            "transposed_gmres_its": st["gmres_its_total"], "recomputed_steps": st["recomputed_steps"],
            "misfit": float(((counts - truth) ** 2).sum().item()),
            "grad_nu": [float(x) for x in grad_nu],
            "grad_g_norm": float(grad_g.norm().item())}


def batch_bench(sk, torch, args):
    """Ensemble leg: independent realistic-type instances of uneven size
    (log-uniform 50k-400k nodes, ~9.3M nodes in all) with their own
    transmission and diffusion rates, stepped together as one block-diagonal
    system (per-instance Newton and GMRES in lockstep, one-level RAS with
    ~1000-node subdomains, overlap 2).  FP32 subdomain factors: FP64 ones
    would take ~255 GB of the 288 GB."""
    import numpy as np
    import seird_inputs as si
    t = time.perf_counter()
    log(f"[bench] building the ensemble of {args.batch_instances} instances")
    bc = si.config_batch(n_inst=args.batch_instances)
    t_gen = time.perf_counter() - t
    log(f"[bench] ensemble {bc.name}: {bc.n} nodes, "
        f"{sum(c.n_sub for c in bc.instances)} subdomains ({t_gen:.1f} s)")
    t = time.perf_counter()
    b = sk.Batch([(c.xy, c.tri, c.params, c.part, c.n_sub) for c in bc.instances],
                 overlap=bc.overlap, tile=32, factor_prec=args.batch_prec)
    t_create = time.perf_counter() - t
    # the ensemble's factors are float32 in tile-32 storage (tile 16 would
    # factor in float64 first); its solve width follows the autotuned choice
    # of the realistic leg with the same factor precision, if that was tile 32
    t_, threads = args.tuned.get(args.batch_prec, (32, 256))
    b.precond.set_solve_threads(threads if t_ == 32 else 256)
    b.precond.enable_timing(True)
    info = b.precond.info()
    log(f"[bench] batch created ({t_create:.1f} s): {info}")
    u = torch.tensor(np.concatenate([c.u0 for c in bc.instances]), device="cuda")
    c0 = bc.instances[0]
    kw = dict(tol=c0.newton_tol, max_it=c0.newton_max_it, restart=c0.gmres_restart,
              rtol=c0.gmres_rtol, atol=c0.gmres_atol, dtol=c0.gmres_dtol, pc_reuse=args.pc_reuse)

    def summary(per):
        return (f"newton max {max(p['newton_its'] for p in per)} "
                f"mean {np.mean([p['newton_its'] for p in per]):.2f}, gmres/instance max "
                f"{max(sum(p['gmres_its']) for p in per)} mean "
                f"{np.mean([sum(p['gmres_its']) for p in per]):.1f}, setups {per[0]['pc_setups']}")

    for w in range(args.warmup):
        per = b.step(u, bc.dt, **kw)
        log(f"[bench] batch warmup step {w}: {summary(per)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    allper = []
    for k in range(args.batch_steps):
        per = b.step(u, bc.dt, **kw)
        allper.append(per)
        log(f"[bench] batch step {k}: {summary(per)} t(res/jac/setup/gmres)ms="
            f"{per[0]['t_residual_ms']:.0f}/{per[0]['t_jacobian_ms']:.0f}/"
            f"{per[0]['t_setup_ms']:.0f}/{per[0]['t_gmres_ms']:.0f}")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ras_ms = sum(p[0]["t_ras_kernel_ms"] for p in allper)
    ras_n = sum(p[0]["n_ras_launches"] for p in allper)
    ras_bytes = allper[0][0]["ras_bytes_per_launch"] if allper else 0.0
    roof = None
    if ras_n > 0:
        achieved = ras_bytes / (ras_ms / ras_n / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_band_solve (subdomain solves of one RAS apply, FP32 factors)",
                "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "avg_launch_ms": ras_ms / ras_n,
                "launches": ras_n, "bytes_per_launch": ras_bytes}
    sizes = [c.n for c in bc.instances]
    return {"metric": "ensemble implicit steps/s (every instance advanced one step)",
            "value": args.batch_steps / sec, "unit": "steps/s",
            "instance_steps_per_s": len(sizes) * args.batch_steps / sec,
            "unknowns": 5 * bc.n, "ms_per_step": 1e3 * sec / args.batch_steps,
            "steps": args.batch_steps,
            "workload": (f"{bc.name}: {len(sizes)} seeded realistic-type instances of "
                         f"{min(sizes)}-{max(sizes)} nodes ({5 * bc.n} unknowns), beta and nu_c "
                         f"x U(0.7,1.3) per instance, dt 1 day, Newton tol {c0.newton_tol}, "
                         f"GMRES({c0.gmres_restart}) rtol {c0.gmres_rtol}, one-level RAS "
                         f"{sum(c.n_sub for c in bc.instances)} subdomains overlap {bc.overlap}, "
                         f"factor_prec {args.batch_prec}, pc_reuse {args.pc_reuse}"),
            "newton_its_max": [max(p["newton_its"] for p in per) for per in allper],
            "gmres_its_per_instance_max": [max(sum(p["gmres_its"]) for p in per) for per in allper],
            "gmres_its_per_instance_mean": [float(np.mean([sum(p["gmres_its"]) for p in per]))
                                            for per in allper],
            "roofline": roof, "precond": info, "solve_threads": threads if t_ == 32 else 256,
            "generate_s": t_gen, "create_s": t_create}


def cpu_baseline(args):
    """The oracle as it stands, timed on the host on a bounded sample."""
    import numpy as np
    import seird_inputs as si
    from oracle import fem, krylov, newton
    # same nesting depth and subdomain size, 32x fewer base nodes
    cfg = si.config_realistic(n_base=max(40, args.n_base // 32), n_ref=args.n_ref,
                              n_sub=max(1, args.n_sub // 32))
    geo = fem.Geometry(cfg.xy, cfg.tri)
    ls = krylov.make_linsolve(geo, cfg.part, cfg.n_sub, cfg.overlap,
                              coarse=(cfg.coarse_parents, cfg.coarse_n),
                              restart=cfg.gmres_restart, rtol=cfg.gmres_rtol)
    t0 = time.perf_counter()
    u1, info = newton.newton_step(cfg.u0, cfg.dt, geo, cfg.params, tol=cfg.newton_tol, linsolve=ls)
    dt = time.perf_counter() - t0
    full_unknowns = 5 * args.full_nodes
    steps_per_s = (1.0 / dt) * (5 * cfg.n) / full_unknowns
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        blas_threads = None
    return {"value": steps_per_s, "unit": "steps/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"first implicit step of a {cfg.n}-node ({5 * cfg.n} unknowns) nested "
                       f"polygon mesh of the same kind ({cfg.n_sub} subdomains of the same size, "
                       f"two-grid RAS, subdomain sparse LU), {dt:.2f} s, Newton its "
                       f"{info['newton_its']}; steps/s scaled to {full_unknowns} unknowns by the "
                       f"unknown ratio (linear-cost assumption)"),
            "host_threads_available": threads, "blas_threads": blas_threads,
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["realistic", "small"], default="realistic")
    ap.add_argument("--prec", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--no-compare-prec", dest="compare_prec", action="store_false",
                    help="skip the FP32/BF16-factor legs")
    ap.add_argument("--tile", default="auto", choices=["auto", "16", "32"],
                    help="tile size of the subdomain band storage (auto: chosen by the autotuner)")
    ap.add_argument("--solve-threads", type=int, default=256, choices=[256, 512, 1024],
                    help="subdomain-solve workgroup size when --tile is given")
    ap.add_argument("--n-base", type=int, default=3900)
    ap.add_argument("--n-ref", type=int, default=4)
    ap.add_argument("--n-sub", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="timed steps of the ensemble leg (0: skip)")
    ap.add_argument("--batch-instances", type=int, default=48)
    ap.add_argument("--batch-prec", type=int, default=1, choices=[0, 1, 2])
    ap.add_argument("--pc-reuse", type=int, default=100,
                    help="Newton iterations a preconditioner setup is reused for (0: fresh every time)")
    ap.add_argument("--adjoint-steps", type=int, default=10,
                    help="implicit steps of the adjoint-gradient measurement (0: skip)")
    ap.add_argument("--adjoint-full", action="store_true",
                    help="measure the gradient on the ~2M-node, 60-step differentiation workload")
    args = ap.parse_args()
    if args.tile != "auto":
        args.tile = int(args.tile)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path "
              "is not part of this build", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import torch
    import paper_2208_01839_amd as sk

    t = time.perf_counter()
    cfg, coarse = build_workload(args)
    args.full_nodes = cfg.n
    log(f"[bench] workload {cfg.name}: {cfg.n} nodes, {len(cfg.tri)} triangles, "
        f"{cfg.n_sub} subdomains, coarse {cfg.coarse_n} nodes ({time.perf_counter() - t:.1f} s)")
    args.tuned = {}
    res = run_steps(sk, torch, cfg, coarse, args.prec, args.steps, args.warmup, args.tile, args.pc_reuse,
                    args.solve_threads)
    args.tuned[args.prec] = (res["tile"], res["solve_threads"])
    sec = res["seconds"]
    stats = res["stats"]
    value = args.steps / sec
    ras_ms = sum(s["t_ras_kernel_ms"] for s in stats)
    ras_n = sum(s["n_ras_launches"] for s in stats)
    ras_bytes = stats[0]["ras_bytes_per_launch"] if stats else 0.0
    roofline = None
    if ras_n > 0:
        avg_s = ras_ms / ras_n / 1e3
        achieved = ras_bytes / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": "k_band_solve (subdomain solves of one RAS apply)",
                    "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS,
                    "traffic": MEASURED_SOLVE_TRAFFIC.get((args.prec, res["tile"], res["solve_threads"])),
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "avg_launch_ms": ras_ms / ras_n, "launches": ras_n,
                    "bytes_per_launch": ras_bytes}
    phase = {k: sum(s[k] for s in stats) / max(1, len(stats)) for k in
             ("t_residual_ms", "t_jacobian_ms", "t_setup_ms", "t_gmres_ms")}
    out = {
        "metric": "SEIRD implicit steps/s at 5M DOF: FP64 vs mixed RAS; adjoint grads/s",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "f64 (f32 subdomain factors)", 2: "f64 (bf16 subdomain factors)"}[args.prec],
        "data": "synthetic",
        "config": {"workload": (f"{cfg.name}: seeded star polygon ~600x400 km, {cfg.n} P1 nodes "
                                f"({5 * cfg.n} unknowns), {len(cfg.tri)} triangles, lognormal density "
                                f"+ 12 urban peaks, dt {cfg.dt} day, Newton tol {cfg.newton_tol}, "
                                f"GMRES({cfg.gmres_restart}) rtol {cfg.gmres_rtol}, "
                                + (f"two-grid RAS {cfg.n_sub} subdomains overlap {cfg.overlap}, coarse "
                                   f"{cfg.coarse_n} nodes" if coarse else
                                   f"one-level RAS {cfg.n_sub} subdomains overlap {cfg.overlap}")),
                   "unknowns": 5 * cfg.n, "tile": res["tile"], "solve_threads": res["solve_threads"],
                   "factor_prec": args.prec,
                   "pc_reuse": args.pc_reuse},
        "newton_its": [s["newton_its"] for s in stats],
        "pc_setups": [s["pc_setups"] for s in stats], "pc_reuse": args.pc_reuse,
        "gmres_its": [s["gmres_its"] for s in stats],
        "phase_ms_per_step": phase,
        "precond": res["info"],
        "autotune": res["tune"],
        "roofline": roofline,
    }
    if args.compare_prec:
        mixed = {}
        for p in (1, 2):
            r2 = run_steps(sk, torch, cfg, coarse, p, args.steps, args.warmup, args.tile, args.pc_reuse,
                           args.solve_threads)
            args.tuned[p] = (r2["tile"], r2["solve_threads"])
            mixed[{1: "fp32", 2: "bf16"}[p]] = {
                "steps_per_s": args.steps / r2["seconds"],
                "speedup_vs_fp64": (args.steps / r2["seconds"]) / value,
                "gmres_its": [s["gmres_its"] for s in r2["stats"]],
                "max_rel_diff_vs_fp64": float(((r2["u"] - res["u"]).abs().max()
                                               / res["u"].abs().max()).item()),
                "tile": r2["tile"], "solve_threads": r2["solve_threads"],
                "phase_ms_per_step": {k: sum(st[k] for st in r2["stats"]) / max(1, len(r2["stats"])) for k in
                                      ("t_residual_ms", "t_jacobian_ms", "t_setup_ms", "t_gmres_ms")},
            }
        out["mixed"] = mixed
    if args.batch_steps > 0:
        del res
        torch.cuda.empty_cache()
        out["batch"] = batch_bench(sk, torch, args)
        torch.cuda.empty_cache()
    if args.adjoint_steps > 0 or args.adjoint_full:
        out["adjoint"] = adjoint_bench(sk, torch, args, cfg, coarse)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on its bounded sample")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
