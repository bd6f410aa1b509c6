"""Full-size shell (1,001,830 Q1 hexahedra, 8,014,640 DoFs, Bueno-Orovio,
five STR R-tree levels) with the 8-column solver and the matrix-core
Chebyshev step: sampled operator rows against the oracle's row assembly,
per-column solve residuals, and time steps of the 8 stimulus-site
simulations against the single-column stepper and, column by column, against
the oracle's step on sampled cells; the same for the single-column stepper."""
import time

import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from oracle.assemble import assemble
from oracle.ionic import gate_step, ionic_current
from workloads.configs import iapp_nodal

pytestmark = pytest.mark.gpu
R = 8


@pytest.fixture(scope="module")
def c4():
    need_gpu()
    pr = make_problem("c4")
    say("c4 full set-up (mixed, 8 columns, mfma)")
    t0 = time.time()
    h, s = problem.build(pr, precision="mixed", max_rhs=R, mfma=True)
    print("c4 set-up s", time.time() - t0, s.info()["t_setup"], flush=True)
    return pr, h, s


def test_c4_levels_and_sampled_rows(c4):
    pr, h, s = c4
    info = s.info()
    assert info["n_cells"][0] == pr["n_cells"] == 1001830
    assert info["n_levels"] == 5
    ratios = [info["n_cells"][l] / info["n_cells"][l + 1] for l in range(4)]
    print("c4 levels", info["n_cells"], "ratios", ratios, "C_op", info["op_complexity"], flush=True)
    assert all(7.0 <= q <= 8.5 for q in ratios)
    rng = np.random.default_rng(12)
    cells = rng.choice(pr["n_cells"], 16, replace=False)
    M, A = assemble(pr, row_cells=cells)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    X = rng.standard_normal((pr["N"], R))
    ref = (cM * M + A) @ X
    rows = (cells[:, None] * pr["b"] + np.arange(pr["b"])).ravel()
    Y = torch.empty(pr["N"] * R, dtype=torch.float64, device="cuda")
    say("c4 sampled apply_multi fp64")
    api.apply_multi(s, 0, dev(X.ravel()), Y, "fp64")
    assert rel(host(Y).reshape(-1, R)[rows], ref[rows]) <= 1e-13
    say("c4 sampled apply_multi fp32")
    api.apply_multi(s, 0, dev(X.ravel()), Y, "mixed")
    assert rel(host(Y).reshape(-1, R)[rows], ref[rows]) <= 5e-6


def test_c4_pcg_multi_residuals(c4):
    pr, h, s = c4
    N = pr["N"]
    B = np.random.default_rng(13).standard_normal((N, R))
    B[:, 4] = 0.0
    b = dev(B.ravel())
    x = torch.zeros(N * R, dtype=torch.float64, device="cuda")
    say("c4 pcg_multi mixed")
    stats = api.pcg_solve_multi(s, b, x, tol=1e-8)
    print("c4 pcg its", [c["its"] for c in stats], flush=True)
    assert all(c["converged"] for c in stats) and stats[4]["its"] == 0
    Ax = torch.empty_like(x)
    api.apply_multi(s, 0, x, Ax, "fp64")
    res = (b - Ax).reshape(N, R)
    for c in range(R):
        if c != 4:
            assert float(torch.linalg.norm(res[:, c])) <= 1.5e-8 * stats[c]["r0"], c


def test_c4_time_steps_multi_vs_single(c4):
    pr, h, s = c4
    N, S = pr["N"], pr["S"]
    U0 = np.zeros(N * R)
    W0 = np.repeat(pr["W0"].reshape(S, N)[:, :, None], R, axis=2).ravel()
    st = api.State(dev(U0), dev(U0), dev(W0), dev(W0),
                   torch.empty(N * R, dtype=torch.float64, device="cuda"))
    ia = np.zeros((N, R))
    for c in range(R):
        ia[np.repeat(pr["stim_masks"][c], pr["b"]), c] = pr["stim_amp"]
    iam = dev(ia.ravel())
    ia0 = dev(ia[:, 0])
    s1 = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(N, dtype=torch.float64, device="cuda"))
    # every column against the oracle's step on sampled cells: 6 from each
    # column's stimulus site and 16 anywhere
    rng = np.random.default_rng(29)
    picks = [rng.choice(pr["n_cells"], 16, replace=False)]
    for c in range(R):
        sc = np.nonzero(pr["stim_masks"][c])[0]
        if len(sc):
            picks.append(rng.choice(sc, min(6, len(sc)), replace=False))
    cells = np.unique(np.concatenate(picks))
    rows = (cells[:, None] * pr["b"] + np.arange(pr["b"])).ravel()
    M, A = assemble(pr, row_cells=cells)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    A0 = (cM * M + A).tocsr()
    M = M.tocsr()
    cc = pr["chi"] * pr["Cm"]
    its = []
    for k in range(3):
        t = (k + 1) * pr["dt"]
        Un, Unm1 = host(st.U).reshape(N, R), host(st.Uprev).reshape(N, R)
        Wn = host(st.W).reshape(S, N, R)[:, rows]
        Wnm1 = host(st.Wprev).reshape(S, N, R)[:, rows]
        say("c4 time_step_multi", k)
        r = api.time_step_multi(s, st, t, iapp=iam, tol=1e-8)
        assert all(c["converged"] for c in r)
        its.append([c["its"] for c in r])
        Unew = host(st.U).reshape(N, R)
        Wg = host(st.W).reshape(S, N, R)[:, rows]
        for c in range(R):
            ustar = 2.0 * Un[rows, c] - Unm1[rows, c]
            Wnew = gate_step(pr["model"], pr["params"], ustar, Wn[:, :, c], Wnm1[:, :, c], pr["dt"], 2)
            g = ionic_current(pr["model"], pr["params"], ustar, Wnew)
            f = np.zeros(N)
            f[rows] = cc / (2.0 * pr["dt"]) * (4.0 * Un[rows, c] - Unm1[rows, c]) - pr["chi"] * g + ia[rows, c]
            bn = (M @ f)[rows]
            assert np.abs(Wg[:, :, c] - Wnew).max() <= 1e-12 * max(1.0, np.abs(Wnew).max())
            q = float(np.linalg.norm(bn - (A0 @ Unew[:, c])[rows]) / np.linalg.norm(bn))
            assert q <= 1e-7, (k, c, q)
        say("c4 time_step single", k)
        r1 = api.time_step(s, s1, t, iapp=ia0, tol=1e-8)
        assert r1["converged"]
    U = host(st.U).reshape(N, R)
    u1 = host(s1.U)
    print("c4 its per step and column", its, flush=True)
    assert np.isfinite(U).all()
    # column 0 is the apex simulation: same problem as the single-column run,
    # both solved to relative residual 1e-8
    assert rel(U[:, 0], u1) <= 1e-5
    # each simulation is excited at its own site only
    for c in range(R):
        cells = np.nonzero(pr["stim_masks"][c])[0]
        if len(cells):
            assert U.reshape(-1, pr["b"], R)[cells, :, c].mean() > 0.0
    assert np.abs(U[:, 0] - U[:, 1]).max() > 0.0


def test_c4_time_steps_against_oracle_rows(c4):
    """Single-column mixed solver, 3 time steps of the apex simulation (section
    3.1 step).  On 64 seeded cells (half of them stimulated): the gates equal the oracle's pointwise BDF2
    gate step at U* = 2 U_n - U_{n-1} (1e-12), and the new U solves the
    oracle's system there: the sampled rows of b_n - A_0 U_{n+1}, with the
    load vector b_n and A_0 assembled by the oracle from the step's inputs,
    stay at the PCG's residual level (a wrong load-vector term or operator
    entry would leave them of the order of b_n)."""
    pr, _, _ = c4
    N, S, b = pr["N"], pr["S"], pr["b"]
    # half of the cells in the stimulated region (where b_n is not zero in
    # the first steps), half anywhere
    rng = np.random.default_rng(17)
    stim = np.nonzero(pr["stim_mask"])[0]
    cells = np.unique(np.concatenate([rng.choice(stim, min(32, len(stim)), replace=False),
                                      rng.choice(pr["n_cells"], 32, replace=False)]))
    rows = (cells[:, None] * b + np.arange(b)).ravel()
    M, A = assemble(pr, row_cells=cells)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    A0 = (cM * M + A).tocsr()
    M = M.tocsr()
    say("c4 single-column set-up (mixed)")
    _, s = problem.build(pr, precision="mixed")
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(N, dtype=torch.float64, device="cuda"))
    c = pr["chi"] * pr["Cm"]
    for k in range(3):
        t = (k + 1) * pr["dt"]
        Un, Unm1 = host(st.U), host(st.Uprev)
        Wn = host(st.W).reshape(S, N)[:, rows]
        Wnm1 = host(st.Wprev).reshape(S, N)[:, rows]
        ia = iapp_nodal(pr, t)
        say("c4 single-column step", k)
        r = api.time_step(s, st, t, iapp=dev(ia) if ia.any() else None, tol=1e-8)
        assert r["converged"]
        ustar = 2.0 * Un[rows] - Unm1[rows]
        Wnew = gate_step(pr["model"], pr["params"], ustar, Wn, Wnm1, pr["dt"], 2)
        g = ionic_current(pr["model"], pr["params"], ustar, Wnew)
        f = np.zeros(N)
        f[rows] = c / (2.0 * pr["dt"]) * (4.0 * Un[rows] - Unm1[rows]) - pr["chi"] * g + ia[rows]
        bn = (M @ f)[rows]
        Wg = host(st.W).reshape(S, N)[:, rows]
        assert np.abs(Wg - Wnew).max() <= 1e-12 * max(1.0, np.abs(Wnew).max())
        res = bn - (A0 @ host(st.U))[rows]
        q = float(np.linalg.norm(res) / np.linalg.norm(bn))
        print(f"c4 step {k}: its={r['its']} sampled |b - A0 U| / |b| = {q:.2e}", flush=True)
        assert q <= 1e-7
