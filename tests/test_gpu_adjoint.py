"""GPU discrete adjoint (torch.autograd.Function over the time stepper)
against the FP64 oracle adjoint and against central finite differences of
the GPU forward loss."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd.adjoint import sensor_misfit_loss
from workloads import make_problem
from oracle.adjoint import AdjointProblem, make_targets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _setup(n, steps, seed=4):
    pr = make_problem("c5", n=n)
    targets = make_targets(pr, steps, pr["s_true"])
    s = np.exp(0.1 * np.random.default_rng(seed).standard_normal(pr["n_cells"]))
    return pr, targets, s


@pytest.mark.parametrize("n,steps,ck", [(16, 7, 3), (32, 12, 5)])
def test_adjoint_matches_oracle(n, steps, ck):
    pr, targets, s = _setup(n, steps)
    ap = AdjointProblem(pr, targets, steps, tol=1e-13, checkpoint=ck)
    loss_ref, grad_ref = ap.gradient(s)
    st = torch.tensor(s, dtype=torch.float64, device="cuda", requires_grad=True)
    say("adjoint vs oracle", n, steps, ck)
    loss = sensor_misfit_loss(st, pr, dev(targets), steps, tol=1e-13, checkpoint=ck)
    loss.backward()
    assert abs(loss.item() - loss_ref) <= 1e-10 * loss_ref
    assert rel(host(st.grad), grad_ref) <= 1e-8


def test_adjoint_matches_finite_differences():
    pr, targets, s = _setup(16, 8)
    tg = dev(targets)
    st = torch.tensor(s, dtype=torch.float64, device="cuda", requires_grad=True)
    say("adjoint gradient c5 16")
    loss = sensor_misfit_loss(st, pr, tg, 8, tol=1e-13, checkpoint=4)
    loss.backward()
    g = host(st.grad)
    rng = np.random.default_rng(2607)
    h = 1e-6
    for k in range(16):
        d = rng.standard_normal(pr["n_cells"])
        d /= np.linalg.norm(d)
        say("fd direction", k)
        lp = sensor_misfit_loss(torch.tensor(s + h * d, device="cuda"), pr, tg, 8).item()
        lm = sensor_misfit_loss(torch.tensor(s - h * d, device="cuda"), pr, tg, 8).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-5 * np.abs(g).sum() / np.sqrt(len(g)) + 1e-5 * abs(fd), (k, fd, g @ d)
