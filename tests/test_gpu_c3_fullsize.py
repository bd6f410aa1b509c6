"""Full-size 64^3 Q2 cube (7,077,888 DoFs, Bueno-Orovio, four agglomerated
levels, 13,824-DoF coarse problem factorised on the device): sampled operator
rows against the oracle's row assembly, solve properties that hold at any size,
and a few time steps with the corner stimulus."""
import time

import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from workloads.configs import iapp_nodal
from oracle.assemble import assemble

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    need_gpu()
    pr = make_problem("c3")
    say("c3 full set-up (mixed)")
    t0 = time.time()
    h, s = problem.build(pr, precision="mixed")
    print("c3 set-up s", time.time() - t0, s.info()["t_setup"], flush=True)
    return pr, h, s


def test_c3_levels_and_sampled_rows(c3):
    pr, h, s = c3
    info = s.info()
    assert info["n_cells"] == [262144, 32768, 4096, 512]
    assert info["n_dofs"] == 7077888
    rng = np.random.default_rng(10)
    cells = rng.choice(pr["n_cells"], 16, replace=False)
    M, A = assemble(pr, row_cells=cells)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    x = rng.standard_normal(pr["N"])
    ref = (cM * M + A) @ x
    rows = (cells[:, None] * pr["b"] + np.arange(pr["b"])).ravel()
    y = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
    say("c3 sampled apply fp64")
    api.apply(s, 0, dev(x), y, "fp64")
    assert rel(host(y)[rows], ref[rows]) <= 1e-13
    say("c3 sampled apply fp32")
    api.apply(s, 0, dev(x), y, "mixed")
    assert rel(host(y)[rows], ref[rows]) <= 5e-6


def test_c3_solve_residual_property(c3):
    pr, h, s = c3
    b = dev(np.random.default_rng(11).standard_normal(pr["N"]))
    x = torch.zeros(pr["N"], dtype=torch.float64, device="cuda")
    say("c3 pcg mixed")
    st = api.pcg_solve(s, b, x, tol=1e-8)
    print("c3 pcg", st, flush=True)
    assert st["converged"] and st["its"] <= 40
    Ax = torch.empty_like(x)
    api.apply(s, 0, x, Ax, "fp64")
    assert float(torch.linalg.norm(b - Ax)) <= 1.5e-8 * st["r0"]


def test_c3_time_steps(c3):
    pr, h, s = c3
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(pr["N"], dtype=torch.float64, device="cuda"))
    its = []
    for k in range(3):
        t = (k + 1) * pr["dt"]
        say("c3 time step", k)
        r = api.time_step(s, st, t, iapp=dev(iapp_nodal(pr, t)), tol=1e-8)
        assert r["converged"]
        its.append(r["its"])
    u = host(st.U)
    print("c3 its", its, "U range", u.min(), u.max(), flush=True)
    # stimulus raises the potential only in and near the stimulated corner
    assert u.max() > 0.0 and np.isfinite(u).all()
