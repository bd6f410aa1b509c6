"""GPU time stepping (ionic update + ICI load vector + warm-started PCG)
against the FP64 oracle stepper, FP64 and mixed precision."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from workloads.configs import iapp_nodal
from oracle.stepper import Simulation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def gpu_run(pr, steps, tol, precision="fp64", lam=None):
    h, s = problem.build(pr, precision=precision, lam_override=lam)
    N, S = pr["N"], pr["S"]
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()),
                   dev(pr["W0"].ravel()), torch.empty(N, dtype=torch.float64, device="cuda"))
    hist, its = [], []
    for k in range(steps):
        t = (k + 1) * pr["dt"]
        ia = iapp_nodal(pr, t)
        stt = api.time_step(s, st, t, iapp=dev(ia) if ia.any() else None, tol=tol)
        assert stt["converged"]
        its.append(stt["its"])
        hist.append(host(st.U).copy())
    return hist, its, host(st.W).reshape(S, N)


CASES = [("c1", None, 10, 1e-10), ("c2", 32, 10, 1e-8), ("c3", 8, 5, 1e-8),
         ("c2", 24, 6, 1e-8)]


@pytest.mark.parametrize("name,n,steps,tol", CASES)
def test_fp64_time_series_matches_oracle(name, n, steps, tol):
    pr = make_problem(name, n=n) if n else make_problem(name)
    sim = Simulation(pr)
    # parity mode: tight tolerance, identical Chebyshev intervals
    _, ref, stats = sim.run(steps, 1e-12, iapp_fn=lambda t: iapp_nodal(pr, t))
    say("time_step fp64", name, n, steps)
    hist, its, W = gpu_run(pr, steps, 1e-12, "fp64", lam=sim.mg.lam)
    for k in range(steps):
        assert rel(hist[k], ref[k]) <= 1e-10, k
    assert [abs(a - s["its"]) <= 1 for a, s in zip(its, stats)] == [True] * steps


@pytest.mark.parametrize("name,n,steps,tol", CASES[:3])
def test_production_tolerance_and_mixed_precision(name, n, steps, tol):
    pr = make_problem(name, n=n) if n else make_problem(name)
    sim = Simulation(pr)
    _, ref, stats = sim.run(steps, 1e-13, iapp_fn=lambda t: iapp_nodal(pr, t))
    for prec in ("fp64", "mixed"):
        say("time_step", prec, name, n, steps, tol)
        hist, its, W = gpu_run(pr, steps, tol, prec)
        err = max(rel(hist[k], ref[k]) for k in range(steps))
        print(f"{name} {prec}: its={its} max rel err vs oracle={err:.2e}")
        # a solve stopped at relative residual tol lands within ~kappa*tol
        assert err <= 1e3 * tol


def test_phase_timing_of_a_step():
    """dgmg_set_phase_timing / dgmg_step_phase_ms: three positive phase
    durations per timed step whose sum stays within the step's wall time, an
    error before any step is timed, and the same trajectory with the events
    on as without them."""
    import time
    from paper_2602_16312_amd import _ffi as F
    pr = make_problem("c2", n=32)
    _, s = problem.build(pr, precision="mixed")
    _, s2 = problem.build(pr, precision="mixed")
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()),
                   dev(pr["W0"].ravel()), torch.empty(pr["N"], dtype=torch.float64, device="cuda"))
    st2 = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()),
                    dev(pr["W0"].ravel()), torch.empty(pr["N"], dtype=torch.float64, device="cuda"))
    api.set_phase_timing(s, True)
    with pytest.raises(F.DGMGError) as e:
        api.step_phase_ms(s)
    assert e.value.code == -1
    for k in range(3):
        t = (k + 1) * pr["dt"]
        say("phase timing step", k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.time_step(s, st, t, tol=1e-8)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        ph = api.step_phase_ms(s)
        assert r["converged"]
        assert all(v > 0 for v in ph.values()), ph
        assert sum(ph.values()) <= wall_ms * 1.05 + 0.05, (ph, wall_ms)
        r2 = api.time_step(s2, st2, t, tol=1e-8)
        assert r2["its"] == r["its"]
        assert torch.equal(st.U, st2.U)
    api.set_phase_timing(s, False)
    with pytest.raises(F.DGMGError):
        api.step_phase_ms(s)


def test_checkpoint_resume_is_bitwise(tmp_path):
    """A run stopped after 4 steps, saved with State.save and resumed by a
    fresh solver from State.load, ends on the same U as an uninterrupted run,
    bit for bit (a time step is a pure function of its state)."""
    pr = make_problem("c2", n=32)
    steps, stop = 8, 4

    def fresh():
        _, s = problem.build(pr, precision="mixed")
        st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()),
                       dev(pr["W0"].ravel()), torch.empty(pr["N"], dtype=torch.float64, device="cuda"))
        return s, st

    s, st = fresh()
    for k in range(steps):
        api.time_step(s, st, (k + 1) * pr["dt"], tol=1e-8)
    U_ref = st.U.clone()
    s, st = fresh()
    for k in range(stop):
        api.time_step(s, st, (k + 1) * pr["dt"], tol=1e-8)
    path = tmp_path / "state.pt"
    st.save(path, step=stop)
    del s, st
    say("resume from checkpoint")
    s, _ = fresh()
    st, meta = api.State.load(path)
    assert meta["step"] == stop
    for k in range(meta["step"], steps):
        r = api.time_step(s, st, (k + 1) * pr["dt"], tol=1e-8)
        assert r["converged"]
    assert torch.equal(st.U, U_ref)
