"""Pins of the oracle's SIPDG assembly on distorted hexahedra (section 3,
forms a_h and m_h on a hexahedral mesh with trilinear geometry).

The meshes are a jittered unit cube (boundary vertices slide within their
planar face, so the domain stays [0,1]^3) and a small jittered voxel shell
(surface vertices fixed, so the domain is the union of the voxels).  Interior
faces of both are curved bilinear surfaces.  Every expected value below comes
from code written here, not from the assembler:

* the exact measure of the domain;
* the energy of linear fields (jumps vanish, so face terms drop out);
* the consistency term, from the exact vector area of a bilinear face,
  S_F = int_F n dS = (x10 - x01) x (x11 - x00) / 2 (diagonals x00-x11 and
  x10-x01);
* the penalty term, from the face's area element |x_s x x_t| and unit normal
  computed from tangent cross products at the face's Gauss points (the
  assembler uses J^-T and Nanson's formula);
* the L2 convergence rate of a manufactured solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workloads import make_problem
from oracle.assemble import assemble

# reference nodes of the Lagrange basis (Gauss-Lobatto; equispaced for p <= 2)
_NODES = {1: np.array([0.0, 1.0]), 2: np.array([0.0, 0.5, 1.0])}


def _cube(n, p, jit=0.2, seed=5):
    return make_problem("c3", n=n, p=p, jitter=jit, seed=seed, group=[])


def _shell(h=0.09):
    return make_problem("c4", h=h)


def _trilinear(X, r):
    """Points of cells with corners X [nc, 8, 3] at reference points r [m, 3]."""
    w = np.ones((r.shape[0], 8))
    for c in range(8):
        for k in range(3):
            w[:, c] *= r[:, k] if (c >> k) & 1 else 1.0 - r[:, k]
    return np.einsum("mc,ncd->nmd", w, X)


def _nodes(pr):
    t = _NODES[pr["p"]]
    q = len(t)
    r = np.array([(t[a], t[b], t[c]) for c in range(q) for b in range(q) for a in range(q)])
    return _trilinear(pr["xyz"][pr["cell_vtx"]], r)          # [nc, b, 3]


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _volumes(X):
    """Exact cell volumes: det J of a trilinear map has degree <= 2 per
    variable, so a 3-point Gauss rule is exact."""
    g, w = _gauss(3)
    tot = np.zeros(X.shape[0])
    for a in range(3):
        for b in range(3):
            for c in range(3):
                xi = np.array([g[a], g[b], g[c]])
                J = np.zeros((X.shape[0], 3, 3))
                for cc in range(8):
                    bits = [(cc >> k) & 1 for k in range(3)]
                    f = [xi[k] if bits[k] else 1.0 - xi[k] for k in range(3)]
                    df = [1.0 if bits[k] else -1.0 for k in range(3)]
                    for k in range(3):
                        prod = df[k] * np.prod([f[m] for m in range(3) if m != k])
                        J[:, :, k] += prod * X[:, cc, :]
                tot += w[a] * w[b] * w[c] * np.linalg.det(J)
    return tot


def _face_pairs(cells):
    """Interior faces by hashing corner sets: (plus, minus, axis) with the
    plus cell seeing the face at xi_axis = 1."""
    seen = {}
    out = []
    for K in range(cells.shape[0]):
        for ax in range(3):
            for side in (0, 1):
                cs = [c for c in range(8) if ((c >> ax) & 1) == side]
                key = tuple(sorted(cells[K, cs]))
                if key in seen:
                    K2, ax2, side2 = seen.pop(key)
                    assert ax2 == ax and side2 != side
                    out.append((K, K2, ax) if side == 1 else (K2, K, ax))
                else:
                    seen[key] = (K, ax, side)
    return np.array(out, dtype=np.int64)


def _face_corners(X, ax):
    """(x00, x10, x01, x11) of the plus cell's xi_ax = 1 face, tangential
    axes m1 < m2 as (s, t)."""
    m1, m2 = [m for m in range(3) if m != ax]
    sel = lambda s, t: (1 << ax) | (s << m1) | (t << m2)
    return X[:, sel(0, 0)], X[:, sel(1, 0)], X[:, sel(0, 1)], X[:, sel(1, 1)]


def _domain_measure(pr):
    if pr.get("kind") == "shell":
        return pr["n_cells"] * pr["h"] ** 3
    return 1.0


MESHES = [("cube p1", lambda: _cube(4, 1)), ("cube p2", lambda: _cube(3, 2)),
          ("shell p1", lambda: _shell())]


@pytest.mark.parametrize("label,mk", MESHES)
def test_measure_kernel_and_symmetry(label, mk):
    pr = mk()
    M, A = assemble(pr)
    one = np.ones(pr["N"])
    assert abs(one @ (M @ one) - _domain_measure(pr)) < 1e-13 * max(1.0, _domain_measure(pr))
    assert abs(_volumes(pr["xyz"][pr["cell_vtx"]]).sum() - _domain_measure(pr)) < 1e-12
    assert np.abs(A @ one).max() < 1e-15 * abs(A).max() * 10
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()


@pytest.mark.parametrize("label,mk", MESHES)
def test_linear_field_energy(label, mk):
    """u = c.x, w = e.x lie in the mapped space and have no jumps, so
    w^T A u = e^T D c |Omega| for a constant tensor D."""
    pr = mk()
    D = np.array([[1.1, 0.1, -0.2], [0.1, 0.9, 0.05], [-0.2, 0.05, 0.6]])
    pr["D_cell"] = np.tile([D[0, 0], D[0, 1], D[0, 2], D[1, 1], D[1, 2], D[2, 2]], (pr["n_cells"], 1))
    _, A = assemble(pr)
    x = _nodes(pr).reshape(-1, 3)
    c, e = np.array([0.7, -1.2, 0.4]), np.array([-0.3, 0.5, 1.1])
    u, w = x @ c, x @ e
    vol = _domain_measure(pr)
    assert abs(u @ (A @ u) - c @ D @ c * vol) < 1e-12 * vol
    assert abs(w @ (A @ u) - e @ D @ c * vol) < 1e-12 * vol


@pytest.mark.parametrize("label,mk", MESHES)
def test_consistency_term_uses_exact_face_vector_areas(label, mk):
    """Continuous linear u, piecewise constant v: cell terms and the penalty
    vanish, leaving v^T A u = -sum_F (v+ - v-) (mean(D+, D-) c) . S_F with
    S_F the exact vector area of the curved face, oriented out of K+."""
    pr = mk()
    rng = np.random.default_rng(21)
    nc = pr["n_cells"]
    # a different SPD tensor per cell
    Lr = rng.standard_normal((nc, 3, 3)) * 0.3 + np.eye(3)
    Dm = np.einsum("nij,nkj->nik", Lr, Lr)
    pr["D_cell"] = np.stack([Dm[:, 0, 0], Dm[:, 0, 1], Dm[:, 0, 2], Dm[:, 1, 1], Dm[:, 1, 2],
                             Dm[:, 2, 2]], axis=1)
    _, A = assemble(pr)
    c = np.array([0.3, -0.8, 0.5])
    u = _nodes(pr).reshape(-1, 3) @ c
    vK = rng.standard_normal(nc)
    v = np.repeat(vK, pr["b"])
    X = pr["xyz"][pr["cell_vtx"]]
    F = _face_pairs(pr["cell_vtx"])
    expect = 0.0
    cen = X.mean(axis=1)
    for ax in range(3):
        f = F[F[:, 2] == ax]
        x00, x10, x01, x11 = _face_corners(X[f[:, 0]], ax)
        S = 0.5 * np.cross(x10 - x01, x11 - x00)
        # orient out of the plus cell
        sgn = np.sign(np.einsum("fd,fd->f", S, cen[f[:, 1]] - cen[f[:, 0]]))
        assert np.all(sgn != 0)
        S = S * sgn[:, None]
        flux = 0.5 * np.einsum("fab,b->fa", Dm[f[:, 0]] + Dm[f[:, 1]], c)
        expect -= ((vK[f[:, 0]] - vK[f[:, 1]]) * np.einsum("fa,fa->f", flux, S)).sum()
    got = v @ (A @ u)
    assert abs(got - expect) <= 1e-12 * max(abs(expect), 1e-3), (got, expect)


@pytest.mark.parametrize("label,mk", MESHES)
def test_penalty_term_on_curved_faces(label, mk):
    """Piecewise constant u, v: only the penalty term remains,
    v^T A u = sum_F (u+ - u-)(v+ - v-) int_F sigma dS with
    sigma = eta_F mean(n^T D+ n, n^T D- n) pointwise and
    eta_F = c p(p+1) mean(|F|/|K+|, |F|/|K-|) (c the configured factor), |F|
    and the integral taken with
    the (p+1)-point Gauss rule on the face (the discrete definition),
    the normal and area element from tangent cross products."""
    pr = mk()
    p = pr["p"]
    D = np.array([[1.4, 0.2, 0.1], [0.2, 0.5, -0.15], [0.1, -0.15, 0.8]])
    pr["D_cell"] = np.tile([D[0, 0], D[0, 1], D[0, 2], D[1, 1], D[1, 2], D[2, 2]], (pr["n_cells"], 1))
    M, A = assemble(pr)
    rng = np.random.default_rng(22)
    nc = pr["n_cells"]
    uK, vK = rng.standard_normal(nc), rng.standard_normal(nc)
    u, v = np.repeat(uK, pr["b"]), np.repeat(vK, pr["b"])
    X = pr["xyz"][pr["cell_vtx"]]
    vol = _volumes(X)
    F = _face_pairs(pr["cell_vtx"])
    g, w = _gauss(p + 1)
    expect = 0.0
    for ax in range(3):
        f = F[F[:, 2] == ax]
        x00, x10, x01, x11 = _face_corners(X[f[:, 0]], ax)
        area = np.zeros(len(f))
        nDn = np.zeros(len(f))
        for a in range(p + 1):
            for bq in range(p + 1):
                s_, t_ = g[a], g[bq]
                xs = (x10 - x00) * (1 - t_) + (x11 - x01) * t_
                xt = (x01 - x00) * (1 - s_) + (x11 - x10) * s_
                cr = np.cross(xs, xt)
                dA = np.linalg.norm(cr, axis=1)
                nh = cr / dA[:, None]
                area += w[a] * w[bq] * dA
                nDn += w[a] * w[bq] * dA * np.einsum("fa,ab,fb->f", nh, D, nh)
        cfac = pr["penalty"][1] if len(pr["penalty"]) > 1 else 1.0
        eta = cfac * p * (p + 1) * 0.5 * (area / vol[f[:, 0]] + area / vol[f[:, 1]])
        expect += ((uK[f[:, 0]] - uK[f[:, 1]]) * (vK[f[:, 0]] - vK[f[:, 1]]) * eta * nDn).sum()
    got = v @ (A @ u)
    assert abs(got - expect) <= 1e-12 * abs(expect), (got, expect)


@pytest.mark.parametrize("p,ns", [(1, [4, 8, 16]), (2, [4, 8])])
def test_manufactured_solution_rate_on_jittered_hexes(p, ns):
    """(c M + A) u = M f with u = cos(pi x) cos(pi y) cos(pi z) (zero normal
    derivative on the cube's faces) and f = (c + 3 pi^2 s) u on jittered
    cubes: the L2 error decays at rate p + 1."""
    s, c = 1.0, 1.0
    fn = lambda y: np.cos(np.pi * y[..., 0]) * np.cos(np.pi * y[..., 1]) * np.cos(np.pi * y[..., 2])
    errs = []
    for n in ns:
        pr = _cube(n, p, jit=0.2, seed=7)
        pr["D_cell"] = np.tile([s, 0.0, 0.0, s, 0.0, s], (pr["n_cells"], 1))
        M, A = assemble(pr)
        x = _nodes(pr).reshape(-1, 3)
        rhs = M @ ((c + 3 * np.pi ** 2 * s) * fn(x))
        U = spla.spsolve((c * M + A).tocsc(), rhs)
        # L2 error with a 5-point rule per direction (own evaluation)
        g, w = _gauss(5)
        r = np.array([(g[a], g[b_], g[cc]) for cc in range(5) for b_ in range(5) for a in range(5)])
        wr = np.array([w[a] * w[b_] * w[cc] for cc in range(5) for b_ in range(5) for a in range(5)])
        t = _NODES[p]
        q = len(t)
        # tensor Lagrange values at r
        L1 = lambda xx: np.stack([np.prod([(xx - t[m]) / (t[j] - t[m]) for m in range(q) if m != j], axis=0)
                                  for j in range(q)], axis=-1)
        Lx, Ly, Lz = L1(r[:, 0]), L1(r[:, 1]), L1(r[:, 2])
        phi = np.einsum("ma,mb,mc->mcba", Lx, Ly, Lz).reshape(len(r), -1)
        X = pr["xyz"][pr["cell_vtx"]]
        xq = _trilinear(X, r)
        eps = 1e-6
        # |det J| at r by central differences of the trilinear map (exact for
        # a polynomial of degree 1 in each variable)
        J = np.stack([(_trilinear(X, r + eps * np.eye(3)[k]) - _trilinear(X, r - eps * np.eye(3)[k])) / (2 * eps)
                      for k in range(3)], axis=-1)
        dJ = np.abs(np.linalg.det(J))
        uh = np.einsum("mi,ni->nm", phi, U.reshape(pr["n_cells"], -1))
        errs.append(np.sqrt((wr[None] * dJ * (uh - fn(xq)) ** 2).sum()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.15, (rates, errs)
