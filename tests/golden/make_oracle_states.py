"""Write the oracle's reference states of the precision workload's nested
instance: the seeded realistic recipe (star polygon, lognormal density with
urban peaks, Ontario rates, dt = 1 day) on a base mesh of 121 nodes refined
four times (32,217 nodes, 161,085 unknowns; 32x fewer nodes than the full
1M-node mesh, same refinement depth), stepped 30 days by the oracle's
coupled Newton with sparse direct solves, over-converged (scaled residual
<= 1e-13 every step).  Stored: the states after steps 1 and 30 and the
Newton counts.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_oracle_states.py  # ~10-20 min on one core
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import seird_inputs as si  # noqa: E402
from oracle import fem, newton  # noqa: E402

N_BASE, N_REF, N_SUB, STEPS, TOL = 121, 4, 32, 30, 1e-13
OUT = os.path.join(HERE, "oracle_polygon32217_r30.npz")


def main():
    cfg = si.config_realistic(n_base=N_BASE, n_ref=N_REF, n_sub=N_SUB)
    geo = fem.Geometry(cfg.xy, cfg.tri)
    u = cfg.u0.copy()
    keep, its = {}, []
    t0 = time.time()
    for k in range(1, STEPS + 1):
        u, info = newton.newton_step(u, cfg.dt, geo, cfg.params, tol=TOL, max_it=30)
        its.append(info["newton_its"])
        if k in (1, 30):
            keep[f"u{k}"] = u.copy()
        print(f"step {k}: newton {info['newton_its']} res {info['res_hist'][-1]:.2e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    np.savez(OUT, n_nodes=cfg.n, n_base=N_BASE, n_ref=N_REF, steps=STEPS, tol=TOL, dt=cfg.dt,
             newton_its=np.array(its), **keep)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
