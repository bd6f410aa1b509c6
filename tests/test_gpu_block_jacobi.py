"""Cell-block Jacobi variant of the Chebyshev smoother (section 6 smoother
with the cells' inverted b x b diagonal blocks as D) against the oracle's
block variant: the V-cycle as an operator on every fine layout and block
size (FP64 and mixed precision), PCG solves, a time series, and the
device set-up path."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from workloads.configs import iapp_nodal
from oracle.assemble import system_matrix
from oracle.hierarchy import build_hierarchy as oracle_hierarchy
from oracle.mg import VCycle, pcg
from oracle.stepper import Simulation

pytestmark = pytest.mark.gpu

CASES = [("c1", dict(n=32)),                       # 2D Q1, b = 4
         ("c2", dict(n=32)),                       # 2D Q2 jittered, b = 9
         ("c2", dict(n=16, p=3, group=[4])),       # b = 16
         ("c3", dict(n=4)),                        # 3D Q2 boxes, b = 27 (matrix-free level 0)
         ("c4", dict(h=0.09))]                     # 3D Q1 shell, STR agglomerates, b = 8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _oracle(pr):
    b = (pr["p"] + 1) ** pr["dim"]
    A0 = system_matrix(pr)[0]
    return A0, VCycle(A0, oracle_hierarchy(pr)["P"], jacobi="cell_block", b=b)


@pytest.mark.parametrize("name,kw", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_vcycle_cell_block(name, kw):
    pr = make_problem(name, **kw)
    A0, mg = _oracle(pr)
    r = np.random.default_rng(21).standard_normal(pr["N"])
    ref = mg(r)
    layouts = ["auto", "axis_ell", "tile_ell"] if pr["p"] >= 2 and name == "c3" else ["auto", "tile_ell"]
    for layout in layouts:
        for prec, tol in (("fp64", 1e-11), ("mixed", 2e-5)):
            h, s = problem.build(pr, precision=prec, lam_override=mg.lam, fine_layout=layout,
                                 jacobi="cell_block")
            z = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
            say("vcycle cell_block", name, kw, layout, prec)
            api.vcycle(s, dev(r), z)
            assert rel(host(z), ref) <= tol, (layout, prec)


@pytest.mark.parametrize("degree,sweeps", [(1, 2), (2, 1), (4, 2)])
def test_vcycle_cell_block_smoother_settings(degree, sweeps):
    """Degree 1 (pending correction through the residual kernel) and other
    degrees and sweep counts with the block variant."""
    pr = make_problem("c2", n=16)
    A0 = system_matrix(pr)[0]
    mg = VCycle(A0, oracle_hierarchy(pr)["P"], degree=degree, sweeps=sweeps, jacobi="cell_block", b=9)
    r = np.random.default_rng(22).standard_normal(pr["N"])
    ref = mg(r)
    for prec, tol in (("fp64", 1e-11), ("mixed", 2e-5)):
        h, s = problem.build(pr, precision=prec, lam_override=mg.lam, cheb_degree=degree,
                             cheb_sweeps=sweeps, jacobi="cell_block")
        z = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
        say("vcycle cell_block settings", degree, sweeps, prec)
        api.vcycle(s, dev(r), z)
        assert rel(host(z), ref) <= tol, (degree, sweeps, prec)


@pytest.mark.parametrize("name,kw", [CASES[1], CASES[3]], ids=["c2", "c3"])
def test_pcg_cell_block(name, kw):
    """PCG with the block-Jacobi V-cycle: iterations and solution against the
    oracle's PCG with the same preconditioner; the library's own Lanczos
    estimates (host and device set-up) give the oracle's interval."""
    pr = make_problem(name, **kw)
    A0, mg = _oracle(pr)
    rng = np.random.default_rng(23)
    b = rng.standard_normal(pr["N"])
    x0 = 0.1 * rng.standard_normal(pr["N"])
    xr, sr = pcg(A0, b, x0, mg, 1e-12)
    for where in ("host", "device"):
        h, s = problem.build(pr, precision="fp64", setup=where, jacobi="cell_block")
        info = s.info()
        for l in range(info["n_levels"] - 1):
            assert abs(info["lam_hi"][l] - mg.lam[l][1]) <= 1e-10 * mg.lam[l][1], (where, l)
        x = dev(x0)
        say("pcg cell_block", name, where)
        st = api.pcg_solve(s, dev(b), x, tol=1e-12)
        assert st["converged"]
        assert abs(st["its"] - sr["its"]) <= 1
        assert rel(host(x), xr) <= 1e-10
    h, s = problem.build(pr, precision="mixed", jacobi="cell_block")
    x = dev(x0)
    say("pcg cell_block mixed", name)
    st = api.pcg_solve(s, dev(b), x, tol=1e-10)
    assert st["converged"]
    assert np.linalg.norm(b - A0 @ host(x)) <= 1.5e-10 * st["r0"]


def test_time_series_cell_block():
    """Mixed-precision time steps with the block smoother reach the oracle's
    time series within the solver tolerance."""
    pr = make_problem("c2", n=16)
    steps = 4
    _, ref, _ = Simulation(pr).run(steps, 1e-12, iapp_fn=lambda t: iapp_nodal(pr, t))
    h, s = problem.build(pr, precision="mixed", jacobi="cell_block")
    N = pr["N"]
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(N, dtype=torch.float64, device="cuda"))
    for k in range(steps):
        t = (k + 1) * pr["dt"]
        say("time step cell_block", k)
        res = api.time_step(s, st, t, iapp=dev(iapp_nodal(pr, t)), tol=1e-10)
        assert res["converged"]
    assert rel(host(st.U), ref[-1]) <= 1e3 * 1e-10
