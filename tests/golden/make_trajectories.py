"""Writes FP64 oracle trajectories for the full-size parity tests, with the
oracle only (parity mode: PCG to relative residual 1e-12, the oracle's own
Chebyshev intervals stored so that the library can take the same ones):

* c2_trajectory.json: the 256x256 jittered Q2 Aliev-Panfilov problem over
  its 100 time steps;
* c3_trajectory.json: the Bueno-Orovio cube at 32^3 Q2 with the corner
  stimulus over 5 time steps.

Per step: ||U_n||_2, the projection w . U_n on a seeded unit vector
(workloads.configs.probe_vector, seed 2610), the PCG iteration count; at some
steps U_n at 512 seeded DoFs (seed 2611).

Usage: python tests/golden/make_trajectories.py c2|c3
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import make_problem  # noqa: E402
from workloads.configs import iapp_nodal, probe_vector  # noqa: E402
from oracle.stepper import Simulation  # noqa: E402

TOL = 1e-12
CASES = {
    "c2": dict(args=("c2",), kw={}, steps=100, sample_steps=[1, 2, 5, 10, 20, 50, 100]),
    "c3": dict(args=("c3",), kw={"n": 32}, steps=5, sample_steps=[1, 2, 3, 4, 5]),
}


def main(name):
    case = CASES[name]
    t0 = time.time()
    pr = make_problem(*case["args"], **case["kw"])
    sim = Simulation(pr)
    print("set-up", time.time() - t0, flush=True)
    w = probe_vector(pr["N"], 2610)
    idx = np.sort(np.random.default_rng(2611).choice(pr["N"], 512, replace=False))
    state = (pr["U0"].copy(), pr["U0"].copy(), pr["W0"].copy(), pr["W0"].copy())
    norms, proj, its, samples = [], [], [], {}
    for n in range(1, case["steps"] + 1):
        t = n * pr["dt"]
        state, st = sim.step(state, t, TOL, iapp_nodal(pr, t))
        U = state[0]
        norms.append(float(np.linalg.norm(U)))
        proj.append(float(w @ U))
        its.append(int(st["its"]))
        if n in case["sample_steps"]:
            samples[str(n)] = U[idx].tolist()
        print(n, its[-1], norms[-1], time.time() - t0, flush=True)
    out = dict(source="FP64 oracle (oracle/stepper.py), PCG to relative residual 1e-12",
               problem=name, overrides=case["kw"], steps=case["steps"], tol=TOL,
               lam=[list(map(float, l)) for l in sim.mg.lam], probe_seed=2610,
               sample_seed=2611, sample_idx=idx.tolist(), norms=norms, proj=proj, its=its,
               samples=samples)
    with open(os.path.join(HERE, f"{name}_trajectory.json"), "w") as f:
        json.dump(out, f)
    print("done", time.time() - t0)


if __name__ == "__main__":
    main(sys.argv[1])
