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


def _corner_map(X, r):
    """Bilinear image of reference points r [m, 2] in cells with corners X [nc, 4, 2]."""
    w = np.stack([(1 - r[:, 0]) * (1 - r[:, 1]), r[:, 0] * (1 - r[:, 1]),
                  (1 - r[:, 0]) * r[:, 1], r[:, 0] * r[:, 1]], axis=1)
    return np.einsum("mc,ncd->nmd", w, X)


@pytest.mark.parametrize("p", [1, 2])
def test_sensor_functional_reproduces_fields(p):
    """e_k^T U (the loss's evaluation functional) on nodal interpolants:
    a Q_p polynomial of the sensor cell's reference coordinates is recovered
    exactly at the sensor's reference point, and a linear physical field
    c.x at the mapped point F_K(xi_k)."""
    from oracle.adjoint import sensor_matrix
    pr = make_problem("c5", n=8, p=p)
    E = sensor_matrix(pr)
    t = np.linspace(0.0, 1.0, p + 1)                    # Lobatto nodes for p <= 2
    ref = np.array([(t[a], t[b]) for b in range(p + 1) for a in range(p + 1)])
    rng = np.random.default_rng(41)
    C = rng.standard_normal((pr["n_cells"], p + 1, p + 1))
    q = lambda K, xi: sum(C[K, a, b] * xi[..., 0] ** a * xi[..., 1] ** b
                          for a in range(p + 1) for b in range(p + 1))
    U = np.concatenate([q(K, ref) for K in range(pr["n_cells"])])
    sc, sr = pr["sensor_cell"], pr["sensor_ref"]
    want = np.array([q(K, r) for K, r in zip(sc, sr)])
    assert np.abs(E @ U - want).max() <= 1e-13 * np.abs(want).max()
    X = pr["xyz"][pr["cell_vtx"]]
    c = np.array([0.8, -1.3])
    U2 = (_corner_map(X, ref) @ c).ravel()
    want2 = np.array([_corner_map(X[K:K + 1], r[None])[0, 0] @ c for K, r in zip(sc, sr)])
    assert np.abs(E @ U2 - want2).max() <= 1e-14
