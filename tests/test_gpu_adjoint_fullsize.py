"""Full-size adjoint problem (256x256 Q2 Aliev-Panfilov, 50 steps, 64
sensors, checkpoints every 10 steps): the GPU gradient with respect to the
65,536 cell scalings at s = 1 against the FP64 oracle adjoint (stored by
tests/golden/make_c5_golden.py, oracle only) and against central finite
differences of the GPU forward loss on 16 seeded directions."""
import json
import os

import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, say, torch
from paper_2602_16312_amd.adjoint import sensor_misfit_loss
from workloads import make_problem

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "c5_adjoint.json")


@pytest.fixture(scope="module")
def c5():
    need_gpu()
    if not os.path.exists(GOLD):
        pytest.skip("oracle golden file not generated")
    g = json.load(open(GOLD))
    pr = make_problem("c5")
    return pr, g


def test_fullsize_adjoint_against_oracle_and_fd(c5):
    pr, g = c5
    steps, tol = g["steps"], g["tol"]
    targets = dev(np.array(g["targets"]))
    s = torch.ones(pr["n_cells"], dtype=torch.float64, device="cuda", requires_grad=True)
    say("c5 full adjoint")
    loss = sensor_misfit_loss(s, pr, targets, steps, tol=tol, checkpoint=10)
    loss.backward()
    grad = host(s.grad)
    assert abs(loss.item() - g["loss"]) <= 1e-9 * g["loss"]
    gn = g["grad_norm"]
    assert abs(np.linalg.norm(grad) - gn) <= 1e-8 * gn
    cells = np.array(g["sample_cells"])
    assert np.abs(grad[cells] - np.array(g["grad_at_cells"])).max() <= 1e-8 * gn
    rng = np.random.default_rng(g["dir_seed"])
    h = 1e-6
    ones = np.ones(pr["n_cells"])
    for k in range(16):
        d = rng.standard_normal(pr["n_cells"])
        d /= np.linalg.norm(d)
        gd = float(grad @ d)
        assert abs(gd - g["grad_dot_dirs"][k]) <= 1e-8 * gn
        say("c5 fd direction", k)
        lp = sensor_misfit_loss(torch.tensor(ones + h * d, device="cuda"), pr, targets, steps,
                                tol=tol).item()
        lm = sensor_misfit_loss(torch.tensor(ones - h * d, device="cuda"), pr, targets, steps,
                                tol=tol).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gd) <= 1e-5 * gn, (k, fd, gd)
