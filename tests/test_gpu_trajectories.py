"""Full-size time series against stored FP64 oracle trajectories
(tests/golden/make_trajectories.py, oracle only), in the launch configuration
the benchmark times (hierarchy and set-up on the GPU, torch memory):

* the 256x256 jittered Q2 Aliev-Panfilov problem over its 100 steps;
* the Bueno-Orovio cube at 32^3 Q2 (matrix-free fine level) over 5 steps.

FP64 (parity mode: the oracle's Chebyshev intervals, PCG to 1e-12) must stay
within 1e-10 of the oracle at every step: the norm, a seeded projection and
512 seeded DoFs.  The mixed solver at the production tolerance 1e-8 is
compared with the same FP64 trajectory: each step's solve stops with
||r|| <= 1e-8 ||r_0||, so its error is at most kappa(A_0) 1e-8 ||r_0|| / ||b||
relative per step (kappa(A_0) <= 1e3 here, ||r_0|| / ||b|| <= 1e-1 for the
warm start), accumulated over the steps: 1e-6 relative bounds 100 steps."""
import json
import os

import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from workloads.configs import iapp_nodal, probe_vector

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return json.load(open(os.path.join(GOLDEN, f"{name}_trajectory.json")))


def _series(g, precision, tol, lam):
    pr = make_problem(g["problem"], **g["overrides"])
    h, s = problem.build(pr, precision=precision, lam_override=lam, setup="device",
                         allocator="torch")
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(pr["N"], dtype=torch.float64, device="cuda"))
    w = dev(probe_vector(pr["N"], g["probe_seed"]))
    idx = torch.tensor(g["sample_idx"], device="cuda")
    out = []
    for n in range(1, g["steps"] + 1):
        t = n * pr["dt"]
        ia = iapp_nodal(pr, t)
        r = api.time_step(s, st, t, iapp=dev(ia) if ia.any() else None, tol=tol)
        assert r["converged"], (n, r)
        U = st.U
        out.append((r["its"], float(torch.linalg.norm(U)), float(w @ U),
                    host(U[idx]) if str(n) in g["samples"] else None, float(U.abs().max())))
    return out


def _compare(g, got, bound, its_slack):
    worst = 0.0
    for n, (its, nrm, prj, smp, umax) in enumerate(got, start=1):
        ref_n = g["norms"][n - 1]
        e = max(abs(nrm - ref_n) / ref_n, abs(prj - g["proj"][n - 1]) / ref_n)
        if smp is not None:
            e = max(e, float(np.abs(smp - np.array(g["samples"][str(n)])).max()) / umax)
        worst = max(worst, e)
        assert e <= bound, (n, e)
        if its_slack is not None:
            assert abs(its - g["its"][n - 1]) <= its_slack, (n, its, g["its"][n - 1])
    return worst


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_fp64_series_matches_oracle_trajectory(name):
    need_gpu()
    g = _golden(name)
    say("trajectory fp64", name, g["steps"], "steps")
    worst = _compare(g, _series(g, "fp64", g["tol"], g["lam"]), 1e-10, 1)
    print(f"{name}: worst relative deviation over {g['steps']} FP64 steps {worst:.2e}", flush=True)


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_mixed_series_against_oracle_trajectory(name):
    need_gpu()
    g = _golden(name)
    say("trajectory mixed", name, g["steps"], "steps")
    worst = _compare(g, _series(g, "mixed", 1e-8, None), 1e-6, None)
    print(f"{name}: mixed precision at tol 1e-8, worst relative deviation from the FP64 oracle "
          f"over {g['steps']} steps {worst:.2e}", flush=True)
