"""Set-up on the GPU (fine SIPDG and mass blocks, prolongation blocks,
Galerkin products P^T A P and the Lanczos estimates): every level's blocks,
prolongations and Chebyshev interval and the mass action against the host
set-up and the oracle's assembly and sparse Galerkin products, for every
supported block size, jittered and box meshes and both agglomeration methods;
solves with a device-built hierarchy against the oracle; the full-size shell
and cube against the host set-up."""
import time

import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from test_setup_host import dense_level
from workloads import make_problem
from workloads.configs import iapp_nodal
from oracle.assemble import system_matrix
from oracle.hierarchy import build_hierarchy as oracle_hierarchy
from oracle.mg import VCycle
from oracle.stepper import Simulation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def shell():
    return make_problem("c4", h=0.09)


CASES = [("c1", lambda: make_problem("c1", n=16)),                       # 2D Q1, b = 4
         ("c2", lambda: make_problem("c2", n=16)),                       # 2D Q2 jittered, b = 9
         ("c2p3", lambda: make_problem("c2", n=8, p=3, group=[4])),      # b = 16
         ("c2p4", lambda: make_problem("c2", n=8, p=4, group=[4])),      # b = 25
         ("c3", lambda: make_problem("c3", n=4)),                        # 3D Q2, b = 27
         ("c3p3", lambda: make_problem("c3", n=4, p=3, group=[2])),      # b = 64
         ("shell", shell)]                                               # 3D Q1 STR R-tree, b = 8


def compare_levels(sh, sd, scale_tol=1e-13):
    ih, idv = sh.info(), sd.info()
    # mass blocks (the load vector's operator)
    N = ih["n_dofs"]
    f = np.random.default_rng(8).standard_normal(N)
    bh = torch.empty(N, dtype=torch.float64, device="cuda")
    bd = torch.empty(N, dtype=torch.float64, device="cuda")
    api.mass_apply(sh, dev(f), bh)
    api.mass_apply(sd, dev(f), bd)
    assert rel(host(bd), host(bh)) <= 1e-14
    assert ih["n_cells"] == idv["n_cells"] and ih["n_faces"] == idv["n_faces"]
    L = ih["n_levels"]
    for l in range(L):
        eh, ed = sh.export_level(l), sd.export_level(l)
        assert np.array_equal(eh["face_cells"], ed["face_cells"]), l
        scale = np.abs(eh["diag"]).max()
        err = np.abs(ed["diag"] - eh["diag"]).max()
        if eh["face_blocks"].size:
            err = max(err, np.abs(ed["face_blocks"] - eh["face_blocks"]).max())
        assert err <= scale_tol * scale, (l, err / scale)
        if l + 1 < L:
            assert np.abs(ed["P"] - eh["P"]).max() <= 1e-14, l
    for l in range(L - 1):
        assert abs(idv["lam_hi"][l] - ih["lam_hi"][l]) <= 1e-10 * ih["lam_hi"][l], l
        assert abs(idv["lam_lo"][l] - ih["lam_lo"][l]) <= 1e-10 * ih["lam_lo"][l], l
    return ih, idv


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_device_setup_matches_host_and_oracle(name, make):
    pr = make()
    say("device setup", name)
    h1, sh = problem.build(pr, precision="fp64", setup="host")
    h2, sd = problem.build(pr, precision="fp64", setup="device")
    ih, idv = compare_levels(sh, sd)
    A0 = system_matrix(pr)[0]
    mg = VCycle(A0, oracle_hierarchy(pr)["P"])
    for l in range(idv["n_levels"]):
        Al = dense_level(sd.export_level(l))
        assert abs(Al - mg.A[l]).max() <= 1e-12 * abs(mg.A[l]).max(), l
    for l in range(idv["n_levels"] - 1):
        assert abs(idv["lam_hi"][l] - mg.lam[l][1]) <= 1e-10 * mg.lam[l][1], l


def test_device_setup_cell_scaling_fixed_penalty_and_adjoint():
    """Per-cell conductivity scalings and the fixed penalty on the device
    assembly; with adjoint = 1 the fine blocks come from the host assembly
    (which also forms the conductivity derivatives)."""
    pr = make_problem("c1", n=16)
    sc = np.random.default_rng(12).uniform(0.5, 2.0, pr["n_cells"])
    for adjoint in (False, True):
        say("device setup scaled", adjoint)
        h1, sh = problem.build(pr, precision="fp64", cell_scale=sc, adjoint=adjoint, setup="host")
        h2, sd = problem.build(pr, precision="fp64", cell_scale=sc, adjoint=adjoint, setup="device")
        compare_levels(sh, sd)
    A0 = system_matrix(pr, scale=sc)[0]
    Al = dense_level(sd.export_level(0))
    assert abs(Al - A0).max() <= 1e-12 * abs(A0).max()


@pytest.mark.parametrize("name,make", [CASES[1], CASES[6]], ids=["c2", "shell"])
def test_device_setup_vcycle_and_time_series(name, make):
    pr = make()
    A0 = system_matrix(pr)[0]
    mg = VCycle(A0, oracle_hierarchy(pr)["P"])
    r = np.random.default_rng(4).standard_normal(pr["N"])
    h, s = problem.build(pr, precision="fp64", lam_override=mg.lam, setup="device")
    z = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
    say("device setup vcycle", name)
    api.vcycle(s, dev(r), z)
    assert rel(host(z), mg(r)) <= 1e-11
    # mixed-precision time series: same iterations as the host-built solver,
    # solution within the tolerance ball of the oracle's
    steps = 4
    sim = Simulation(pr)
    _, ref, _ = sim.run(steps, 1e-12, iapp_fn=lambda t: iapp_nodal(pr, t))
    runs = {}
    for where in ("host", "device"):
        h, s = problem.build(pr, precision="mixed", setup=where)
        N = pr["N"]
        st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                       torch.empty(N, dtype=torch.float64, device="cuda"))
        its = []
        for k in range(steps):
            t = (k + 1) * pr["dt"]
            say("device setup time step", name, where, k)
            res = api.time_step(s, st, t, iapp=dev(iapp_nodal(pr, t)), tol=1e-10)
            assert res["converged"]
            its.append(res["its"])
        runs[where] = (its, host(st.U))
    assert runs["device"][0] == runs["host"][0]
    # a solve stopped at relative residual tol lands within ~kappa * tol
    assert rel(runs["device"][1], ref[-1]) <= 1e3 * 1e-10


@pytest.mark.parametrize("name", ["c4", "c3"])
def test_device_setup_full_size(name):
    """The 1.0M-hex shell (Q1, 5 STR levels) and the 64^3 Q2 cube (4 grid
    levels): every coarse level, prolongation and Chebyshev interval of the
    device set-up against the host set-up."""
    pr = make_problem(name)
    out = {}
    for where in ("host", "device"):
        say("full-size set-up", name, where)
        t0 = time.perf_counter()
        h, s = problem.build(pr, precision="mixed", setup=where)
        wall = time.perf_counter() - t0
        info = s.info()
        L = info["n_levels"]
        ex = [s.export_level(l) for l in range(1, L)]
        P = [s.export_level(0, blocks=False)["P"]] + [e["P"] for e in ex[:-1]]
        out[where] = (info, ex, P)
        print(f"{name} {where}: set-up {wall:.2f} s, phases "
              + ", ".join(f"{k} {v:.2f}" for k, v in info["t_setup"].items()))
        del s, h
    (ih, exh, Ph), (idv, exd, Pd) = out["host"], out["device"]
    assert ih["n_cells"] == idv["n_cells"] and ih["n_faces"] == idv["n_faces"]
    for l, (eh, ed) in enumerate(zip(exh, exd), start=1):
        assert np.array_equal(eh["face_cells"], ed["face_cells"]), l
        scale = np.abs(eh["diag"]).max()
        err = max(np.abs(ed["diag"] - eh["diag"]).max(),
                  np.abs(ed["face_blocks"] - eh["face_blocks"]).max() if eh["face_blocks"].size else 0)
        assert err <= 1e-13 * scale, (l, err / scale)
    for l, (a, b) in enumerate(zip(Ph, Pd)):
        assert np.abs(a - b).max() <= 1e-14, l
    for l in range(ih["n_levels"] - 1):
        assert abs(idv["lam_hi"][l] - ih["lam_hi"][l]) <= 1e-10 * ih["lam_hi"][l], l
