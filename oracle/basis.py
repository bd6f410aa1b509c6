"""Reference-element ingredients: Gauss-Lobatto Lagrange basis (section 3,
the tensor-product space Q_p and its Lagrangian basis), Gauss-Legendre
quadrature, and the multilinear geometry map of quad/hex cells.

Pins (tests/test_oracle_basis.py): cardinality, partition of unity, zero-sum
of gradients, exactness of the quadrature for degree <= 2p+1, Jacobian of an
affine cell equals its edge matrix.
"""
import itertools

import numpy as np
from numpy.polynomial import legendre as npleg


def gl_nodes(p):
    """Gauss-Lobatto nodes on [0,1]: the end points plus the roots of the
    derivative of the degree-p Legendre polynomial."""
    inner = npleg.Legendre.basis(p).deriv().roots() if p > 1 else np.array([])
    x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (x + 1.0)


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [0,1] (points, weights)."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(nodes, x):
    """Values and first derivatives of the 1D Lagrange polynomials on
    ``nodes`` at points ``x``: arrays [len(x), len(nodes)]."""
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    val = np.ones((x.size, n))
    der = np.zeros((x.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                val[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
        for k in range(n):
            if k == j:
                continue
            term = np.full(x.size, 1.0 / (nodes[j] - nodes[k]))
            for m in range(n):
                if m != j and m != k:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            der[:, j] += term
    return val, der


def multi_index(p, d):
    """Local DoF i -> (i0, i1[, i2]) with i = i0 + (p+1) i1 + (p+1)^2 i2."""
    q = p + 1
    return np.array([[(i // q ** k) % q for k in range(d)] for i in range(q ** d)])


def tensor_basis(p, d, xi):
    """Q_p Lagrange basis on GL nodes at reference points xi [n, d].

    Returns (phi [n, b], grad [n, b, d]) with b = (p+1)^d.
    """
    xi = np.atleast_2d(xi)
    nodes = gl_nodes(p)
    mi = multi_index(p, d)
    vals, ders = [], []
    for k in range(d):
        v, dv = lagrange_1d(nodes, xi[:, k])
        vals.append(v)
        ders.append(dv)
    n, b = xi.shape[0], mi.shape[0]
    phi = np.ones((n, b))
    for k in range(d):
        phi *= vals[k][:, mi[:, k]]
    grad = np.ones((n, b, d))
    for k in range(d):
        for m in range(d):
            grad[:, :, k] *= (ders[m] if m == k else vals[m])[:, mi[:, m]]
    return phi, grad


def tensor_rule(n, d):
    """Tensor Gauss-Legendre rule with n points per direction on [0,1]^d."""
    x, w = gauss_legendre(n)
    pts = np.array(list(itertools.product(x, repeat=d)))[:, ::-1]
    wts = np.array([np.prod(c) for c in itertools.product(w, repeat=d)])
    return pts.copy(), wts


def corner_shape(d, xi):
    """Multilinear corner functions and their gradients at xi [n, d].

    Corner c = c0 + 2 c1 + 4 c2 sits at reference point (c0, c1, c2).
    Returns (psi [n, 2^d], dpsi [n, 2^d, d]).
    """
    xi = np.atleast_2d(xi)
    n = xi.shape[0]
    nc = 2 ** d
    psi = np.ones((n, nc))
    dpsi = np.ones((n, nc, d))
    for c in range(nc):
        for k in range(d):
            bit = (c >> k) & 1
            f = xi[:, k] if bit else 1.0 - xi[:, k]
            df = 1.0 if bit else -1.0
            psi[:, c] *= f
            for m in range(d):
                dpsi[:, c, m] *= df if m == k else f
    return psi, dpsi


def cell_geometry(X, xi):
    """Geometry of cells with corner coordinates X [nc, 2^d, d] at reference
    points xi [nq, d].

    Returns (x [nc, nq, d], J [nc, nq, d, d] with J[a, k] = dx_a/dxi_k,
    detJ [nc, nq], JinvT [nc, nq, d, d]).
    """
    d = X.shape[2]
    psi, dpsi = corner_shape(d, xi)
    x = np.einsum("qc,ncd->nqd", psi, X)
    J = np.einsum("qck,nca->nqak", dpsi, X)
    detJ = np.linalg.det(J)
    JinvT = np.linalg.inv(J).transpose(0, 1, 3, 2)
    return x, J, detJ, JinvT
