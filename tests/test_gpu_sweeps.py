"""One row of the level / time-step sweeps (the paper's tables of PCG
iterations against the number of levels and against dt) through the same
code path as the benchmark's sweep mode, on a small jittered shell: the
library's iteration count at every step equals the oracle's (same STR
agglomerates, the oracle's Chebyshev intervals)."""
import numpy as np
import pytest

import bench
from gpu_util import need_gpu, say
from workloads import make_problem
from workloads.configs import iapp_nodal
from oracle.stepper import Simulation

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,dt", [(3, 0.05), (4, 0.05), (3, 0.5)])
def test_sweep_row_iterations_match_oracle(L, dt):
    need_gpu()
    pr = make_problem("c4", h=0.09, agglo=("rtree_str", 8, L), dt=dt, steps=6)
    sim = Simulation(pr)
    _, _, stats = sim.run(pr["steps"], 1e-8, iapp_fn=lambda t: iapp_nodal(pr, t))
    ref = [s_["its"] for s_ in stats]
    say("sweep row", L, dt)
    r = bench._its_stats(pr, "fp64", 1e-8, "rel_r0", lam_override=sim.mg.lam)
    got = r["its_per_step"]
    print(f"L={L} dt={dt}: library {got}, oracle {ref}", flush=True)
    assert len(got) == len(ref)
    assert all(abs(a - b) <= 1 for a, b in zip(got, ref))
    assert np.mean(np.array(got) == np.array(ref)) >= 0.8
