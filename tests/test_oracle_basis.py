"""Pins of the oracle's reference-element ingredients (section 3: Q_p
Lagrange basis; quadrature and geometry used by the forms)."""
import json
import os

import numpy as np
import pytest

from oracle.basis import (gl_nodes, gauss_legendre, tensor_basis, tensor_rule,
                          cell_geometry, multi_index)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gl_nodes_closed_form():
    assert np.allclose(gl_nodes(1), [0, 1], atol=1e-15)
    assert np.allclose(gl_nodes(2), [0, 0.5, 1], atol=1e-15)
    s = 1 / np.sqrt(5)
    assert np.allclose(gl_nodes(3), [0, (1 - s) / 2, (1 + s) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("p,d", [(1, 2), (2, 2), (3, 2), (1, 3), (2, 3)])
def test_cardinality_unity_and_gradient_sum(p, d):
    nodes = gl_nodes(p)[multi_index(p, d)]
    phi, _ = tensor_basis(p, d, nodes)
    assert np.allclose(phi, np.eye(phi.shape[0]), atol=1e-13)
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (17, d))
    phi, grad = tensor_basis(p, d, x)
    assert np.allclose(phi.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(grad.sum(axis=1), 0.0, atol=1e-12)


@pytest.mark.parametrize("p,d", [(1, 2), (2, 2), (3, 2), (2, 3)])
def test_basis_gradient_matches_finite_difference(p, d):
    rng = np.random.default_rng(1)
    x = rng.uniform(0.1, 0.9, (5, d))
    _, grad = tensor_basis(p, d, x)
    h = 1e-6
    for k in range(d):
        e = np.zeros(d); e[k] = h
        fd = (tensor_basis(p, d, x + e)[0] - tensor_basis(p, d, x - e)[0]) / (2 * h)
        assert np.allclose(grad[:, :, k], fd, atol=1e-8)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_quadrature_exact_to_degree_2p_plus_1(p):
    for d in (1, 2, 3):
        pts, w = tensor_rule(p + 1, d)
        for deg in range(2 * p + 2):
            exps = [deg] + [2 * p + 1 - (k % 2) for k in range(d - 1)]
            val = (w * np.prod(pts ** np.array(exps)[None, :], axis=1)).sum()
            assert abs(val - np.prod([1.0 / (e + 1) for e in exps])) < 1e-14
    # one degree more is not integrated exactly
    x, wt = gauss_legendre(p + 1)
    assert abs((wt * x ** (2 * p + 2)).sum() - 1.0 / (2 * p + 3)) > 1e-6


def test_affine_cell_jacobian_is_edge_matrix():
    rng = np.random.default_rng(2)
    E = np.array([[0.3, 0.1, 0.0], [-0.05, 0.25, 0.02], [0.0, 0.03, 0.4]])
    o = np.array([0.2, 0.1, -0.3])
    corners = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], float)
    X = (o + corners @ E.T)[None]
    xi = rng.uniform(0, 1, (6, 3))
    x, J, detJ, JinvT = cell_geometry(X, xi)
    assert np.allclose(J[0], E[None], atol=1e-15)
    assert np.allclose(detJ, np.linalg.det(E), atol=1e-15)
    assert np.allclose(x[0], o + xi @ E.T, atol=1e-15)


def test_paper_dof_counts():
    """N = cells * (p+1)^d reproduces every DoF count printed in the paper,
    and coarse agglomerated levels carry (p+1)^d DoFs per agglomerate (the
    Q_p space on the bounding box)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_dof_counts.json")))
    for m in g["fine_meshes"]:
        for p, n in m["dofs"].items():
            b = tensor_basis(int(p), m["dim"], np.zeros((1, m["dim"])))[0].shape[1]
            assert m["cells"] * b == n, m["cite"]
    for h in g["agglomerated_levels"]:
        b = tensor_basis(h["p"], h["dim"], np.zeros((1, h["dim"])))[0].shape[1]
        assert [c * b for c in h["cards"]] == h["dofs"], h["cite"]
