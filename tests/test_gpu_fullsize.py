"""Full-size 256x256 Q2 Aliev-Panfilov problem (589,824 DoFs) in the launch
configuration the benchmark times (hierarchy built on the GPU): FP64 steps
against the oracle, mixed precision against the FP64 oracle, sampled operator
rows of the device-assembled operator."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from oracle.assemble import assemble
from oracle.stepper import Simulation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    need_gpu()
    pr = make_problem("c2")
    sim = Simulation(pr)
    return pr, sim


def _state(pr):
    N = pr["N"]
    return api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()),
                     dev(pr["W0"].ravel()), torch.empty(N, dtype=torch.float64, device="cuda"))


def test_sampled_operator_rows(c2):
    pr, sim = c2
    h, s = problem.build(pr, precision="mixed", setup="device")
    rng = np.random.default_rng(9)
    cells = rng.choice(pr["n_cells"], 64, replace=False)
    M, A = assemble(pr, row_cells=cells)
    A0r = sim.cM * M + A
    x = rng.standard_normal(pr["N"])
    y = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
    say("full c2 sampled apply")
    api.apply(s, 0, dev(x), y, "fp64")
    rows = (cells[:, None] * pr["b"] + np.arange(pr["b"])).ravel()
    ref = (A0r @ x)[rows]
    assert rel(host(y)[rows], ref) <= 1e-13


def test_two_steps_fp64_and_mixed(c2):
    pr, sim = c2
    _, ref, stats = sim.run(2, 1e-12)
    say("full c2 fp64 2 steps")
    h, s = problem.build(pr, precision="fp64", lam_override=sim.mg.lam, setup="device")
    st = _state(pr)
    for k in range(2):
        r = api.time_step(s, st, (k + 1) * pr["dt"], tol=1e-12)
        assert r["converged"]
        assert rel(host(st.U), ref[k]) <= 1e-10
    del s, h
    say("full c2 mixed 2 steps")
    h, s = problem.build(pr, precision="mixed", setup="device")
    st = _state(pr)
    for k in range(2):
        r = api.time_step(s, st, (k + 1) * pr["dt"], tol=1e-8)
        assert r["converged"]
        err = rel(host(st.U), ref[k])
        print(f"mixed step {k}: its={r['its']} rel err vs FP64 oracle={err:.2e}")
        assert err <= 1e-6
