"""Matrix-free fine level on meshes of identical axis-aligned boxes: the
sum-factorised operator against the oracle's assembled A_0 (every block size
the library supports, FP64 and FP32, with per-cell conductivity scalings),
the V-cycle and a time series against the oracle, and the error for meshes
that are not boxes."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from paper_2602_16312_amd._ffi import DGMGError
from workloads import make_problem
from workloads.configs import iapp_nodal
from oracle.assemble import assemble, system_matrix
from oracle.hierarchy import build_hierarchy as oracle_hierarchy
from oracle.mg import VCycle
from oracle.stepper import Simulation

pytestmark = pytest.mark.gpu
MF = dict(fine_layout="matrix_free")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


CASES = [("c3", dict(n=4)), ("c3", dict(n=6, p=1, group=[3])), ("c3", dict(n=4, p=3, group=[2])),
         ("c1", dict(n=16)), ("e1", dict(n=8, p=2, group=[4])), ("e1", dict(n=8, p=3, group=[4])),
         ("e1", dict(n=8, p=4, group=[4]))]


@pytest.mark.parametrize("name,kw", CASES)
def test_apply_matches_oracle(name, kw):
    pr = make_problem(name, **kw)
    scale = np.random.default_rng(3).uniform(0.5, 2.0, pr["n_cells"])
    h, s = problem.build(pr, precision="mixed", cell_scale=scale, **MF)
    assert s.info()["fine_layout"] == "matrix_free"
    M, A = assemble(pr, scale)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    A0 = cM * M + A
    x = np.random.default_rng(1).standard_normal(pr["N"])
    ref = A0 @ x
    y = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
    say("mf apply", name, kw, "fp64")
    api.apply(s, 0, dev(x), y, "fp64")
    assert rel(host(y), ref) <= 1e-13
    say("mf apply", name, kw, "fp32")
    api.apply(s, 0, dev(x), y, "mixed")
    assert rel(host(y), ref) <= 3e-6


@pytest.mark.parametrize("name,kw", [("c3", dict(n=8)), ("e1", dict(n=16, p=2))])
def test_vcycle_matches_oracle(name, kw):
    pr = make_problem(name, **kw)
    A0 = system_matrix(pr)[0]
    mg = VCycle(A0, oracle_hierarchy(pr)["P"])
    r = np.random.default_rng(2).standard_normal(pr["N"])
    ref = mg(r)
    for prec, tol in (("fp64", 1e-11), ("mixed", 2e-5)):
        h, s = problem.build(pr, precision=prec, lam_override=mg.lam, **MF)
        z = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
        say("mf vcycle", name, kw, prec)
        api.vcycle(s, dev(r), z)
        assert rel(host(z), ref) <= tol, prec


def test_time_series_matches_oracle():
    pr = make_problem("c3", n=8)
    steps = 5
    sim = Simulation(pr)
    _, ref, stats = sim.run(steps, 1e-12, iapp_fn=lambda t: iapp_nodal(pr, t))
    h, s = problem.build(pr, precision="fp64", lam_override=sim.mg.lam, **MF)
    N, S = pr["N"], pr["S"]
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(N, dtype=torch.float64, device="cuda"))
    for k in range(steps):
        t = (k + 1) * pr["dt"]
        say("mf time step", k)
        r = api.time_step(s, st, t, iapp=dev(iapp_nodal(pr, t)), tol=1e-12)
        assert r["converged"]
        assert abs(r["its"] - stats[k]["its"]) <= 1
        assert rel(host(st.U), ref[k]) <= 1e-10, k


def test_auto_layout_choice():
    cases = [("c3", dict(n=4), "matrix_free"), ("c1", dict(n=8), "axis_ell"),
             ("c2", dict(n=8), "axis_ell")]
    for name, kw, want in cases:
        pr = make_problem(name, **kw)
        h, s = problem.build(pr)
        assert s.info()["fine_layout"] == want, name
    h, s = problem.build(make_problem("c3", n=4), max_rhs=8)
    assert s.info()["fine_layout"] == "axis_ell"


def test_rejects_meshes_that_are_not_boxes():
    pr = make_problem("c2", n=8)         # jittered
    with pytest.raises(DGMGError):
        problem.build(pr, **MF)
