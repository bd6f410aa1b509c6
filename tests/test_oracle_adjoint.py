"""Pin of the oracle's discrete adjoint: its gradient matches central finite
differences of the oracle's own forward loss (section 3.1 stepper, sensor
misfit over the time series) along random directions."""
import numpy as np
import pytest

from workloads import make_problem
from oracle.adjoint import AdjointProblem, make_targets


@pytest.mark.parametrize("name,n,steps,ck", [("c5", 8, 7, 3), ("c1", 8, 6, 4)])
def test_adjoint_gradient_matches_central_differences(name, n, steps, ck):
    overrides = {}
    if name == "c1":
        overrides = dict(sensors=(16, 11), target_seed=12)
    pr = make_problem(name, n=n, **overrides)
    rng = np.random.default_rng(3)
    s_true = pr["s_true"]
    targets = make_targets(pr, steps, s_true)
    ap = AdjointProblem(pr, targets, steps, tol=1e-14, checkpoint=ck)
    s = np.exp(0.1 * rng.standard_normal(pr["n_cells"]))
    loss, grad = ap.gradient(s)
    assert loss > 0
    h = 1e-5
    for k in range(3):
        d = rng.standard_normal(pr["n_cells"])
        d /= np.linalg.norm(d)
        fd = (ap.forward(s + h * d) - ap.forward(s - h * d)) / (2 * h)
        assert abs(fd - grad @ d) <= 1e-6 * max(abs(fd), np.abs(grad).sum() * 1e-3), (fd, grad @ d)
