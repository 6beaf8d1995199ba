"""Input generators: the ensemble recipe holds what it states."""
import numpy as np

import seird_inputs as si


def test_ensemble_recipe():
    bc = si.config_batch(n_inst=6, n_min=3000, n_max=12000, nodes_per_sub=400, n_ref=1)
    base = si.params_ontario()
    assert len(bc.instances) == 6
    for c in bc.instances:
        # sizes near the log-uniform targets (Delaunay + refinement round them)
        assert 2000 < c.n < 16000
        assert c.part.min() == 0 and c.part.max() == c.n_sub - 1
        assert abs(c.n / c.n_sub - 400) < 150
        p = c.params
        f = p.beta_I / 0.006
        assert 0.7 <= f <= 1.3 and p.beta_E == p.beta_I
        fn = np.array(p.nu[:4]) / np.array(base.nu[:4])
        assert np.all((fn >= 0.7) & (fn <= 1.3)) and p.nu[4] == 0.0
        N = c.u0.sum(1)
        assert N.min() > base.A
        assert c.dt * p.beta_I * N.max() <= 1.0
        # only s and i are seeded
        assert np.all(c.u0[:, [1, 3, 4]] == 0.0)
    # instances differ in size and rates
    assert len({c.n for c in bc.instances}) == 6
    assert len({c.params.beta_I for c in bc.instances}) == 6
