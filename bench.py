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
reported in "mixed", with each field's error at step 30 against the FP64
leg and, on the 32x smaller nested instance of the same recipe, against the
oracle's stored step-30 state.  The ensemble leg ("batch") steps 48 uneven
instances together; the adjoint leg ("adjoint") times one misfit gradient of
the differentiation workload (~2M nodes, 60 daily steps, checkpoints every
10 steps).  The CPU baseline is the FP64 oracle (numpy/scipy) timed on the
host's cores on a bounded sample of the same workload (independent steps
of the nested instance, one per worker process), scaled to 5M unknowns by
the unknown ratio.
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
MEASURED_SOLVE_TRAFFIC = {(0, 32, 256): (20.927 + 0.177) * 1e9, (0, 32, 512): (21.950 + 0.190) * 1e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


FIELDS = ("S", "E", "I", "R", "D")


def per_field_errors(u, ref):
    """Relative error of every compartment: max norm and 2-norm."""
    import numpy as np
    u = np.asarray(u).reshape(-1, 5)
    ref = np.asarray(ref).reshape(-1, 5)
    out = {}
    for c, name in enumerate(FIELDS):
        d, r = u[:, c] - ref[:, c], ref[:, c]
        out[name] = {"linf_rel": float(np.abs(d).max() / max(np.abs(r).max(), 1e-300)),
                     "l2_rel": float(np.linalg.norm(d) / max(np.linalg.norm(r), 1e-300))}
    return out


def build_workload(args):
    import seird_inputs as si
    if args.workload == "small":
        cfg = si.config_small()
        coarse = None
    else:
        cfg = si.config_realistic(n_base=args.n_base, n_ref=args.n_ref, n_sub=args.n_sub)
        coarse = (cfg.coarse_parents, cfg.coarse_n)
    return cfg, coarse


def run_steps(sk, torch, cfg, coarse, prec, steps, warmup, tile, pc_reuse=0, threads=256, until=0, pc_keep=0):
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
              rtol=cfg.gmres_rtol, atol=cfg.gmres_atol, dtol=cfg.gmres_dtol, pc_reuse=pc_reuse,
              pc_keep_steps=pc_keep)
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
    perf = pc.perf(reset=True)
    # untimed steps up to `until` (the precision comparison is at step 30)
    for k in range(warmup + steps, until):
        sk.step(prob, pc, u, cfg.dt, **kw)
    torch.cuda.synchronize()
    return dict(seconds=t1 - t0, stats=stats, info=info, u=u, tile=tile, solve_threads=threads, tune=tune,
                perf=perf, prob=prob, pc=pc, steps_done=max(until, warmup + steps))


def adjoint_bench(sk, torch, args, cfg, coarse):
    """One gradient of the case-count misfit (forward record + reverse
    sweep) with respect to the per-node transmission field and the five
    diffusion coefficients; checkpoints every 10 steps (5 for short runs)."""
    import numpy as np
    import seird_inputs as si
    if args.adjoint == "full":
        t = time.perf_counter()
        cfg = si.config_differentiation()
        coarse = (cfg.coarse_parents, cfg.coarse_n)
        steps, every = cfg.steps, 10
        log(f"[bench] adjoint workload {cfg.name} built ({time.perf_counter() - t:.1f} s)")
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
    prob.set_beta_field(torch.ones(cfg.n, dtype=torch.float64, device="cuda"))

    def gradient(keep, ckpt=every):
        log(f"[bench] adjoint: timed forward record (pc_keep_steps={keep}, checkpoint every {ckpt})")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
        counts = sk.forward_record(prob, pc, u, steps, cfg.dt, region, 40, ckpt_every=ckpt,
                                   pc_keep_steps=keep, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        log(f"[bench] adjoint: forward {t1 - t0:.2f} s; reverse sweep")
        grad_g, grad_nu, st = sk.adjoint(prob, pc, 2 * (counts - truth), rtol=1e-8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        log(f"[bench] adjoint: forward {t1 - t0:.2f} s, reverse {t2 - t1:.2f} s, {st}")
        return counts, grad_g, grad_nu, st, t0, t1, t2

    counts, grad_g, grad_nu, st, t0, t1, t2 = gradient(0)
    kept = None
    if args.keep_steps > 0:
        # the same gradient with setups kept across the steps of each
        # checkpoint segment, forward and in the transposed solves
        _, kg, knu, kst, k0, k1, k2 = gradient(args.keep_steps)
        kept = {"keep_steps": args.keep_steps, "value": 1.0 / (k2 - k0), "unit": "grads/s",
                "forward_s": k1 - k0, "reverse_s": k2 - k1,
                "transposed_gmres_its": kst["gmres_its_total"], "reverse_setups": kst["setups"],
                "grad_g_rel_diff": float((kg - grad_g).norm().item() / grad_g.norm().item()),
                "grad_nu_rel_diff": float(np.abs(knu - grad_nu).max() / np.abs(grad_nu).max())}
    resident = None
    if args.adjoint_resident:
        # every state of the run kept in device memory (one checkpoint
        # segment: 61 states of 5n float64), so the reverse sweep recomputes
        # nothing; setups kept as above
        keep = max(args.keep_steps, 0)
        _, rg, rnu, rst, r0, r1, r2 = gradient(keep, ckpt=steps)
        resident = {"keep_steps": keep, "value": 1.0 / (r2 - r0), "unit": "grads/s",
                    "forward_s": r1 - r0, "reverse_s": r2 - r1, "recomputed_steps": rst["recomputed_steps"],
                    "state_gb": (steps + 1) * 5 * cfg.n * 8 / 1e9,
                    "transposed_gmres_its": rst["gmres_its_total"], "reverse_setups": rst["setups"],
                    "grad_g_rel_diff": float((rg - grad_g).norm().item() / grad_g.norm().item()),
                    "grad_nu_rel_diff": float(np.abs(rnu - grad_nu).max() / np.abs(grad_nu).max())}
    return {"metric": "adjoint gradients/s", "value": 1.0 / (t2 - t0), "unit": "grads/s",
            "workload": (f"{cfg.name}: {cfg.n} nodes ({5 * cfg.n} unknowns), {steps} daily steps, "
                         f"checkpoint every {every}, 40 Voronoi regions, gradient w.r.t. the per-node "
                         f"transmission field and 5 diffusion coefficients, two-grid RAS {cfg.n_sub} "
                         f"subdomains, base transmission beta_I = beta_E = {cfg.params.beta_I}"
                         + (" (0.006 instead of 0.01 keeps dt*beta*g*max N below 1 on this mesh)"
                            if args.adjoint == "full" else "")),
            "forward_s": t1 - t0, "reverse_s": t2 - t1,
            "transposed_gmres_its": st["gmres_its_total"], "recomputed_steps": st["recomputed_steps"],
            "reverse_setups": st["setups"], "kept_setups": kept, "resident_states": resident,
            "misfit": float(((counts - truth) ** 2).sum().item()),
            "grad_nu": [float(x) for x in grad_nu],
            "grad_g_norm": float(grad_g.norm().item())}


def pgs_bench(sk, torch, args, cfg):
    """The paper's decoupled Picard-Gauss-Seidel solver (Appendix A) on the
    realistic workload: one-level RAS over the same 1024 partitions (scalar
    subdomains, overlap 2), sweeps until epsilon (Eq. picardtol) <= 1e-10,
    inner GMRES rtol 1e-5; the coupled residual reached is reported."""
    prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
    pgs = sk.PicardGS(prob, cfg.part, cfg.n_sub, cfg.overlap, tile=32)
    u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
    kw = dict(tol=args.pgs_tol, max_sweeps=60, restart=cfg.gmres_restart, rtol=cfg.gmres_rtol)
    for w in range(args.warmup if args.warmup < 2 else 1):
        st = pgs.step(u, cfg.dt, **kw)
        log(f"[bench] pgs warmup: sweeps {st['sweeps']} gmres {st['gmres_its']} res {st['res_scaled']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.pgs_steps):
        st = pgs.step(u, cfg.dt, **kw)
        stats.append(st)
        log(f"[bench] pgs step {k}: sweeps {st['sweeps']} gmres {st['gmres_its']} res {st['res_scaled']:.2e} "
            f"setup/gmres ms {st['t_setup_ms']:.0f}/{st['t_gmres_ms']:.0f}")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    # the same steps with each compartment's preconditioner set up at the
    # first sweep of a step only (pc_lag), from the same initial state
    u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
    for w in range(args.warmup if args.warmup < 2 else 1):
        pgs.step(u, cfg.dt, pc_lag=True, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lstats = []
    for k in range(args.pgs_steps):
        st = pgs.step(u, cfg.dt, pc_lag=True, **kw)
        lstats.append(st)
        log(f"[bench] pgs (lagged setups) step {k}: sweeps {st['sweeps']} gmres {st['gmres_its']} "
            f"res {st['res_scaled']:.2e} setup/gmres ms {st['t_setup_ms']:.0f}/{st['t_gmres_ms']:.0f}")
    torch.cuda.synchronize()
    lsec = time.perf_counter() - t1
    lagged = {"value": args.pgs_steps / lsec, "unit": "steps/s", "ms_per_step": 1e3 * lsec / args.pgs_steps,
              "sweeps": [st["sweeps"] for st in lstats],
              "gmres_its_per_compartment": [st["gmres_its"] for st in lstats],
              "res_scaled": [st["res_scaled"] for st in lstats],
              "setups_per_step": [st["pc_setups"] for st in lstats],
              "phase_ms_per_step": {"t_setup_ms": sum(st["t_setup_ms"] for st in lstats) / len(lstats),
                                    "t_gmres_ms": sum(st["t_gmres_ms"] for st in lstats) / len(lstats)}}
    return {"metric": "implicit steps/s by Picard-Gauss-Seidel sweeps", "value": args.pgs_steps / sec,
            "unit": "steps/s", "steps": args.pgs_steps, "ms_per_step": 1e3 * sec / args.pgs_steps,
            "workload": (f"{cfg.name}: the realistic workload, decoupled compartments (Appendix A), "
                         f"epsilon tol {args.pgs_tol}, inner GMRES({cfg.gmres_restart}) rtol {cfg.gmres_rtol} "
                         f"with one-level RAS of {cfg.n_sub} scalar subdomains overlap {cfg.overlap}"),
            "sweeps": [st["sweeps"] for st in stats],
            "gmres_its_per_compartment": [st["gmres_its"] for st in stats],
            "res_scaled": [st["res_scaled"] for st in stats],
            "setups_per_step": [st["pc_setups"] for st in stats],
            "phase_ms_per_step": {"t_setup_ms": sum(st["t_setup_ms"] for st in stats) / len(stats),
                                  "t_gmres_ms": sum(st["t_gmres_ms"] for st in stats) / len(stats)},
            "lagged_setups": lagged}


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

    tune = None
    for w in range(args.warmup):
        per = b.step(u, bc.dt, **kw)
        log(f"[bench] batch warmup step {w}: {summary(per)}")
        if w == 0:
            # the solve width chosen on the ensemble itself (its first factors)
            tune = b.autotune(reps=3)
            log(f"[bench] batch autotune: {tune}")
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
                         f"{min(sizes)}-{max(sizes)} nodes ({5 * bc.n} unknowns), beta = 0.006 and "
                         f"nu_c each x U(0.7,1.3) per instance (base 0.006 keeps dt*beta*max N below 1 on "
                         f"every instance), dt 1 day, Newton tol {c0.newton_tol}, "
                         f"GMRES({c0.gmres_restart}) rtol {c0.gmres_rtol}, one-level RAS "
                         f"{sum(c.n_sub for c in bc.instances)} subdomains overlap {bc.overlap}, "
                         f"factor_prec {args.batch_prec}, pc_reuse {args.pc_reuse}"),
            "newton_its_max": [max(p["newton_its"] for p in per) for per in allper],
            "gmres_its_per_instance_max": [max(sum(p["gmres_its"]) for p in per) for per in allper],
            "gmres_its_per_instance_mean": [float(np.mean([sum(p["gmres_its"]) for p in per]))
                                            for per in allper],
            "roofline": roof, "precond": info,
            "solve_threads": tune["solve_threads"] if tune else (threads if t_ == 32 else 256),
            "autotune": tune,
            "generate_s": t_gen, "create_s": t_create}


def _oracle_sample_worker(args_tuple):
    """One worker of the CPU baseline: build the nested sample and time
    ``n_steps`` oracle steps on it (BLAS limited to one thread)."""
    n_base, n_ref, n_sub, n_steps = args_tuple
    import time as _t
    from threadpoolctl import threadpool_limits
    import seird_inputs as si
    from oracle import fem, krylov, newton
    with threadpool_limits(limits=1):
        cfg = si.config_realistic(n_base=n_base, n_ref=n_ref, n_sub=n_sub)
        geo = fem.Geometry(cfg.xy, cfg.tri)
        ls = krylov.make_linsolve(geo, cfg.part, cfg.n_sub, cfg.overlap,
                                  coarse=(cfg.coarse_parents, cfg.coarse_n),
                                  restart=cfg.gmres_restart, rtol=cfg.gmres_rtol)
        u = cfg.u0.copy()
        t0 = _t.perf_counter()
        its = []
        for _ in range(n_steps):
            u, info = newton.newton_step(u, cfg.dt, geo, cfg.params, tol=cfg.newton_tol, linsolve=ls)
            its.append(info["newton_its"])
        return _t.perf_counter() - t0, cfg.n, its


def cpu_baseline(args):
    """The oracle as it stands, timed on the host's cores on a bounded
    sample: every worker process runs ``--cpu-steps`` implicit steps of the
    nested instance of the same recipe (32x fewer nodes, same refinement
    depth and subdomain size, two-grid RAS, subdomain sparse LU) with BLAS
    on one thread; the machine's rate is the sum of the workers' rates,
    scaled to the full workload by the unknown ratio."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:  # pragma: no cover
        avail = os.cpu_count() or 1
    workers = max(1, min(args.cpu_workers, avail))
    job = (max(40, args.n_base // 32), args.n_ref, max(1, args.n_sub // 32), args.cpu_steps)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_sample_worker, [job] * workers)
    wall = time.perf_counter() - t0
    n_sample = res[0][1]
    full_unknowns = 5 * args.full_nodes
    rate = sum(args.cpu_steps / r[0] for r in res)  # sample steps/s over all workers
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    return {"value": rate * (5 * n_sample) / full_unknowns, "unit": "steps/s", "cores": workers,
            "kind": "oracle",
            "sample": (f"{workers} worker processes (one core each, BLAS on one thread), each timing "
                       f"{args.cpu_steps} implicit steps of a {n_sample}-node ({5 * n_sample} unknowns) "
                       f"nested polygon mesh of the same recipe (32x fewer nodes, same subdomain size, "
                       f"two-grid RAS with subdomain sparse LU, Newton tol 1e-10, GMRES rtol 1e-5); "
                       f"step times {', '.join(f'{r[0] / args.cpu_steps:.2f}' for r in res[:4])}"
                       f"{'...' if len(res) > 4 else ''} s; the summed rate is scaled to {full_unknowns} "
                       f"unknowns by the unknown ratio (linear-cost assumption)"),
            "cpu_model": cpu_model, "host_cores_available": avail, "wall_s": wall,
            "newton_its": res[0][2]}


def oracle_precision_leg(sk, torch, args):
    """Precision workload at the nested instance (32x fewer nodes, same
    recipe and refinement depth): 30 daily steps on the GPU with FP64, FP32
    and BF16 subdomain factors, every field's error at step 30 against the
    oracle's stored over-converged state (written by
    tests/golden/make_oracle_states.py), at the workload's tolerances."""
    import numpy as np
    import seird_inputs as si
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "oracle_polygon32217_r30.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    cfg = si.config_realistic(n_base=int(ref["n_base"]), n_ref=int(ref["n_ref"]), n_sub=32)
    coarse = (cfg.coarse_parents, cfg.coarse_n)
    out = {"workload": (f"{cfg.name}: nested instance of the realistic recipe, {cfg.n} nodes "
                        f"({5 * cfg.n} unknowns), 32 subdomains, two-grid RAS, 30 daily steps, Newton "
                        f"tol {cfg.newton_tol}, GMRES rtol {cfg.gmres_rtol}; reference: the oracle's "
                        f"state at step 30 (Newton with direct solves to scaled residual "
                        f"{float(ref['tol'])})")}
    for prec, name in ((0, "fp64"), (1, "fp32"), (2, "bf16")):
        prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
        pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, factor_prec=prec, coarse=coarse)
        u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
        its = []
        for _ in range(int(ref["steps"])):
            st = sk.step(prob, pc, u, cfg.dt, tol=cfg.newton_tol, rtol=cfg.gmres_rtol, pc_reuse=args.pc_reuse)
            its.append(sum(st["gmres_its"]))
        torch.cuda.synchronize()
        out[name] = {"per_field": per_field_errors(u.cpu().numpy(), ref["u30"]), "gmres_its_total": sum(its)}
    return out


PEAK_MFMA_TFLOPS = {0: 78.6, 1: 157.3, 2: 157.3}  # FP64, FP32 (BF16 factors are factored in FP32)


def solve_roofline(stats, prec):
    """The subdomain-solve kernel of a leg: algorithmic bytes per launch
    (factors in the storage precision plus local vectors) over its HIP-event
    time per launch."""
    ras_ms = sum(s["t_ras_kernel_ms"] for s in stats)
    ras_n = sum(s["n_ras_launches"] for s in stats)
    if ras_n <= 0:
        return None
    nbytes = stats[0]["ras_bytes_per_launch"]
    achieved = nbytes / (ras_ms / ras_n / 1e3) / 1e9
    return {"bound": "hbm", "kernel": "k_band_solve (subdomain solves of one RAS apply, "
                                      + {0: "FP64", 1: "FP32", 2: "BF16"}[prec] + " factors)",
            "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "avg_launch_ms": ras_ms / ras_n, "launches": ras_n, "bytes_per_launch": nbytes, "traffic": None}


def factor_roofline(perf, prec):
    """Subdomain factorisation against the matrix-core peak of its
    arithmetic: flops of the tile products per setup over the HIP-event time
    of the factorisation launch, averaged over the timed setups."""
    if not perf or perf["setups"] <= 0:
        return None
    ms = perf["t_lu_ms"] / perf["setups"]
    achieved = perf["lu_mfma_flops"] / (ms * 1e-3) / 1e12
    peak = PEAK_MFMA_TFLOPS[prec]
    return {"bound": "mfma", "kernel": "k_band_lu32 (subdomain LU of one setup, "
                                       + ("FP64" if prec == 0 else "FP32") + " MFMA)",
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "useful_tflops": perf["lu_useful_flops"] / (ms * 1e-3) / 1e12,
            "flops_per_launch": perf["lu_mfma_flops"], "useful_flops_per_launch": perf["lu_useful_flops"],
            "avg_launch_ms": ms, "launches": perf["setups"],
            "extract_ms": perf["t_extract_ms"] / perf["setups"],
            "traffic": None}


def spmv_roofline(sk, torch, prob, u, dt, reps=50):
    """k_spmv on the Jacobian at the final state: algorithmic bytes (the
    node-block matrix once, its index arrays once, x gathered once per node,
    y written) over the HIP-event time per launch on the launch stream."""
    vals = prob.jacobian(u, dt)
    x = torch.randn(prob.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        prob.spmv(vals, x, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        prob.spmv(vals, x, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = prob.n * (25 * 8 + 8 + 40 + 40) + prob.nslots * (10 * 8 + 4)
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "k_spmv (node-block Jacobian times a vector)", "achieved": achieved,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "avg_launch_ms": ms, "launches": reps, "bytes_per_launch": nbytes,
            "traffic": None}


def precond_variants_bench(sk, torch, args, cfg, coarse, direct):
    """The preconditioner variants of Section 3.2 on the realistic workload,
    beside the direct two-grid RAS of the headline (``direct``: its steps/s
    and GMRES counts): two-grid RAS-V2 (coarse system by inner GMRES(30),
    rtol 1e-5, at most 100 iterations, preconditioned by RAS on the coarse
    graph with the fine partition's coarse shares, overlap 1; flexible outer
    GMRES), two-grid RAS-V3 (the same inner GMRES preconditioned by an
    aggregation-AMG V-cycle, one Jacobi sweep each side, last level at most
    40 nodes) and one-level RAS (outer cap 200).  Each starts from the initial
    state after one untimed step, as the headline does."""
    out = {}
    kw = dict(tol=cfg.newton_tol, max_it=cfg.newton_max_it, restart=cfg.gmres_restart,
              rtol=cfg.gmres_rtol, atol=cfg.gmres_atol, dtol=cfg.gmres_dtol, pc_reuse=args.pc_reuse,
              gmres_max_it=200)
    tile, threads = args.tuned.get(0, (32, 256))
    for name in ("two_grid_v2", "two_grid_v3", "one_level"):
        steps = args.variant_steps if name != "one_level" else 1
        prob = sk.Problem(cfg.xy, cfg.tri, cfg.params)
        pc = sk.Precond(prob, cfg.part, cfg.n_sub, cfg.overlap, tile=tile, solve_threads=threads,
                        coarse=coarse if name != "one_level" else None)
        if name == "two_grid_v2":
            pc.set_coarse_krylov(n_sub=0, overlap=1, restart=30, max_it=100, rtol=1e-5)
        if name == "two_grid_v3":
            pc.set_coarse_amg(max_coarse=40, nu=1, omega=2.0 / 3.0, restart=30, max_it=100, rtol=1e-5)
        u = torch.tensor(cfg.u0, dtype=torch.float64, device="cuda")
        st = sk.step(prob, pc, u, cfg.dt, **kw)
        log(f"[bench] {name} warmup: newton {st['newton_its']} gmres {st['gmres_its']}")
        if name != "one_level":
            pc.coarse_krylov_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for k in range(steps):
            st = sk.step(prob, pc, u, cfg.dt, **kw)
            stats.append(st)
            log(f"[bench] {name} step {k}: newton {st['newton_its']} gmres {st['gmres_its']} "
                f"setup/gmres ms {st['t_setup_ms']:.0f}/{st['t_gmres_ms']:.0f}")
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        its = [g for s in stats for g in s["gmres_its"]]
        rec = {"steps": steps, "steps_per_s": steps / sec, "ms_per_step": 1e3 * sec / steps,
               "vs_direct_two_grid": (steps / sec) / direct["value"],
               "newton_its": [s["newton_its"] for s in stats],
               "gmres_its": [s["gmres_its"] for s in stats],
               "mean_gmres_its_per_newton": sum(its) / max(1, len(its)),
               "inexact_solves": sum(s.get("inexact_solves", 0) for s in stats),
               "phase_ms_per_step": {k: sum(s[k] for s in stats) / len(stats)
                                     for k in ("t_setup_ms", "t_gmres_ms")}}
        if name != "one_level":
            ks = pc.coarse_krylov_stats()
            rec["inner"] = {"solves": ks["solves"], "mean_its": ks["its"] / max(1, ks["solves"]),
                            "max_its": ks["its_max"], "capped_at_100": ks["unconverged"]}
            if name == "two_grid_v2":
                rec["inner"]["coarse_subdomains"] = ks["coarse_subdomains"]
            else:
                rec["inner"]["amg_levels"] = ks["amg_levels"]
                rec["inner"]["amg_last_nodes"] = ks["amg_last_nodes"]
        out[name] = rec
        del pc, prob, u
        torch.cuda.empty_cache()
    out["two_grid_direct"] = {"steps_per_s": direct["value"],
                              "mean_gmres_its_per_newton": direct["mean_its"]}
    out["workload"] = (f"{cfg.name}: the headline workload and tolerances; Section 3.2 variants "
                       f"(Table 2 of Section 4.1 compares the same four on a unit square)")
    return out


def model22_bench(sk, torch, args, cfg):
    """The 22-compartment model of Appendix C on the realistic mesh (22
    unknowns per node): compartment-wise Picard-Gauss-Seidel sweeps to
    epsilon 1e-10, the ten diffusing compartments by GMRES(30) rtol 1e-5 with
    one-level RAS of the same 1024 subdomains (scalar, overlap 2)."""
    import seird_inputs as si
    p = si.params22_realistic()
    mesh = sk.Mesh(cfg.xy, cfg.tri)
    t = time.perf_counter()
    model = sk.Model22(mesh, p, cfg.part, cfg.n_sub, cfg.overlap, tile=32)
    log(f"[bench] model22 created ({time.perf_counter() - t:.1f} s)")
    u = torch.tensor(si.state22_from(cfg.u0), dtype=torch.float64, device="cuda")
    kw = dict(tol=1e-10, max_sweeps=64, restart=cfg.gmres_restart, rtol=cfg.gmres_rtol)
    st = model.step(u, cfg.dt, **kw)
    log(f"[bench] model22 warmup: sweeps {st['sweeps']} setups {st['pc_setups']} res {st['res_scaled']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.m22_steps):
        st = model.step(u, cfg.dt, **kw)
        stats.append(st)
        log(f"[bench] model22 step {k}: sweeps {st['sweeps']} gmres {sum(st['gmres_its'])} setups {st['pc_setups']} "
            f"res {st['res_scaled']:.2e} setup/gmres ms {st['t_setup_ms']:.0f}/{st['t_gmres_ms']:.0f}")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    names = si.COMPARTMENTS22
    return {"metric": "implicit steps/s, 22-compartment model", "value": args.m22_steps / sec, "unit": "steps/s",
            "steps": args.m22_steps, "ms_per_step": 1e3 * sec / args.m22_steps,
            "workload": (f"{cfg.name}: {cfg.n} nodes x 22 compartments ({22 * cfg.n} unknowns), dt {cfg.dt} day, "
                         f"Appendix C model with synthetic rates, compartment-wise Picard-Gauss-Seidel to "
                         f"epsilon 1e-10, inner GMRES({cfg.gmres_restart}) rtol {cfg.gmres_rtol} with one-level "
                         f"RAS of {cfg.n_sub} scalar subdomains overlap {cfg.overlap}"),
            "sweeps": [s["sweeps"] for s in stats],
            "gmres_its_per_compartment": [{nm: s["gmres_its"][k] for k, nm in enumerate(names)
                                           if s["gmres_its"][k]} for s in stats],
            "pc_setups": [s["pc_setups"] for s in stats],
            "res_scaled": [s["res_scaled"] for s in stats],
            "phase_ms_per_step": {"t_setup_ms": sum(s["t_setup_ms"] for s in stats) / len(stats),
                                  "t_gmres_ms": sum(s["t_gmres_ms"] for s in stats) / len(stats)}}


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
    ap.add_argument("--solve-threads", type=int, default=256, choices=[256, 128, 512, 1024],
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
    ap.add_argument("--adjoint", choices=["full", "short", "none"], default="full",
                    help="adjoint-gradient leg: the ~2M-node, 60-step differentiation workload "
                         "(full), --adjoint-steps steps of the realistic mesh (short), or none")
    ap.add_argument("--adjoint-steps", type=int, default=10,
                    help="implicit steps of the short adjoint leg")
    ap.add_argument("--no-adjoint-resident", dest="adjoint_resident", action="store_false",
                    help="skip the adjoint variant that keeps every state of the run in device memory "
                         "(no checkpoint recomputation)")
    ap.add_argument("--p-steps", type=int, default=30,
                    help="step at which the precision legs compare their fields (untimed steps are "
                         "added after the timed ones to reach it)")
    ap.add_argument("--pgs-steps", type=int, default=3,
                    help="timed steps of the Picard-Gauss-Seidel leg (0: skip)")
    ap.add_argument("--variant-steps", type=int, default=2,
                    help="timed steps of the two-grid RAS-V2 leg (one-level RAS runs one step; 0: skip both)")
    ap.add_argument("--m22-steps", type=int, default=2,
                    help="timed steps of the 22-compartment leg (0: skip)")
    ap.add_argument("--keep-steps", type=int, default=2,
                    help="FP64 leg, and the adjoint gradient, repeated with each step's preconditioner "
                         "setup kept for this many later steps (0: skip)")
    ap.add_argument("--pgs-tol", type=float, default=1e-10,
                    help="epsilon tolerance of the Picard-Gauss-Seidel sweeps")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="worker processes of the CPU baseline (capped by the cores available)")
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps per CPU-baseline worker")
    args = ap.parse_args()
    if args.tile != "auto":
        args.tile = int(args.tile)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
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
                    args.solve_threads, until=args.p_steps if args.compare_prec else 0)
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
    kernels = [roofline] if roofline else []
    lu = factor_roofline(res["perf"], args.prec)
    if lu:
        kernels.append(lu)
    kernels.append(spmv_roofline(sk, torch, res["prob"], res["u"], cfg.dt))
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
        "roofline_kernels": kernels,
    }
    if args.compare_prec:
        mixed = {}
        for p in (1, 2):
            r2 = run_steps(sk, torch, cfg, coarse, p, args.steps, args.warmup, args.tile, args.pc_reuse,
                           args.solve_threads, until=args.p_steps)
            args.tuned[p] = (r2["tile"], r2["solve_threads"])
            mixed[{1: "fp32", 2: "bf16"}[p]] = {
                "steps_per_s": args.steps / r2["seconds"],
                "speedup_vs_fp64": (args.steps / r2["seconds"]) / value,
                "gmres_its": [s["gmres_its"] for s in r2["stats"]],
                "max_rel_diff_vs_fp64": float(((r2["u"] - res["u"]).abs().max()
                                               / res["u"].abs().max()).item()),
                "per_field_vs_fp64": {"step": r2["steps_done"],
                                      "errors": per_field_errors(r2["u"].cpu().numpy(), res["u"].cpu().numpy())},
                "setup_lu_ms": (r2["perf"]["t_lu_ms"] / r2["perf"]["setups"]) if r2["perf"]["setups"] else None,
                "roofline": solve_roofline(r2["stats"], p),
                "factor_roofline": factor_roofline(r2["perf"], p),
                "tile": r2["tile"], "solve_threads": r2["solve_threads"],
                "phase_ms_per_step": {k: sum(st[k] for st in r2["stats"]) / max(1, len(r2["stats"])) for k in
                                      ("t_residual_ms", "t_jacobian_ms", "t_setup_ms", "t_gmres_ms")},
            }
        log("[bench] precision legs on the nested instance against the oracle's step-30 state")
        mixed["vs_oracle_nested"] = oracle_precision_leg(sk, torch, args)
        out["mixed"] = mixed
    if args.keep_steps > 0:
        # the headline leg again, a setup serving up to 1 + keep_steps steps
        tk, thk = args.tuned.get(0, (32, 256))
        rk = run_steps(sk, torch, cfg, coarse, 0, args.steps, args.warmup, tk, args.pc_reuse, thk,
                       until=res["steps_done"], pc_keep=args.keep_steps)
        out["kept_setups"] = {
            "steps_per_s": args.steps / rk["seconds"], "vs_headline": (args.steps / rk["seconds"]) / value,
            "keep_steps": args.keep_steps,
            "setups_per_step": [st["pc_setups"] for st in rk["stats"]],
            "newton_its": [st["newton_its"] for st in rk["stats"]],
            "gmres_its": [st["gmres_its"] for st in rk["stats"]],
            "max_rel_diff_vs_headline": {"step": rk["steps_done"],
                                         "value": float(((rk["u"] - res["u"]).abs().max()
                                                         / res["u"].abs().max()).item())},
            "phase_ms_per_step": {k: sum(st[k] for st in rk["stats"]) / max(1, len(rk["stats"])) for k in
                                  ("t_residual_ms", "t_jacobian_ms", "t_setup_ms", "t_gmres_ms")},
            "workload": "the headline workload and tolerances; each preconditioner setup made by a step "
                        f"also serves the next {args.keep_steps} steps (rebuilt earlier if its GMRES count "
                        "exceeds twice its fresh count plus 5)"}
        del rk
    if args.variant_steps > 0 and coarse is not None:
        its = [g for st in stats for g in st["gmres_its"]]
        out["precond_variants"] = precond_variants_bench(
            sk, torch, args, cfg, coarse, {"value": value, "mean_its": sum(its) / max(1, len(its))})
    if args.pgs_steps > 0:
        out["pgs"] = pgs_bench(sk, torch, args, cfg)
        out["pgs"]["vs_newton"] = out["pgs"]["value"] / value
        out["pgs"]["lagged_setups"]["vs_newton"] = out["pgs"]["lagged_setups"]["value"] / value
    if args.m22_steps > 0 and args.workload == "realistic":
        out["model22"] = model22_bench(sk, torch, args, cfg)
    if args.batch_steps > 0:
        del res
        torch.cuda.empty_cache()
        out["batch"] = batch_bench(sk, torch, args)
        torch.cuda.empty_cache()
    if args.adjoint != "none":
        out["adjoint"] = adjoint_bench(sk, torch, args, cfg, coarse)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on its bounded sample")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
