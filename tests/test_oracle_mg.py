"""Pins of the oracle's hierarchy, transfers, smoother, V-cycle and PCG
(section 4 agglomeration; section 5.1 inherited operators and
prolongation; section 6 Chebyshev-Jacobi / V-cycle / PCG)."""
import numpy as np
import pytest
import scipy.linalg as sla

from workloads import make_problem
from oracle.assemble import system_matrix
from oracle.basis import gl_nodes, multi_index
from oracle.hierarchy import build_hierarchy, fine_nodes_level0, box_nodes
from oracle.mg import (VCycle, cell_block_inverse, chebyshev, diagonal_blocks, galerkin,
                       lanczos_theta_max, lanczos_theta_max_block, pcg)


@pytest.mark.parametrize("name,n,expect", [("c1", 32, [1024, 64]),
                                           ("c2", 32, [1024, 64, 4]),
                                           ("c3", 8, [512, 64, 8, 1])])
def test_partition_cover_and_nesting(name, n, expect):
    pr = make_problem(name, n=n)
    h = build_hierarchy(pr)
    assert h["n"] == expect
    for l, par in enumerate(h["parents"]):
        assert par.shape[0] == expect[l]
        assert np.array_equal(np.unique(par), np.arange(expect[l + 1]))
        sizes = np.bincount(par)
        assert np.all(sizes == expect[l] // expect[l + 1])
    # every agglomerate's fine cells form a contiguous block of the grid
    ids = h["ids"]
    cen = pr["xyz"][pr["cell_vtx"]].mean(axis=1)
    for l in range(1, len(ids)):
        for K in range(min(expect[l], 5)):
            c = cen[ids[l] == K]
            ext = c.max(axis=0) - c.min(axis=0)
            assert np.all(ext < (expect[0] / expect[l]) ** (1 / pr["dim"]) / n * 1.01)


@pytest.mark.parametrize("name,n", [("c2", 16), ("c3", 4)])
def test_prolongation_reproduces_coarse_polynomials(name, n):
    pr = make_problem(name, n=n)
    h = build_hierarchy(pr)
    p, d = pr["p"], pr["dim"]
    rng = np.random.default_rng(3)
    for l, P in enumerate(h["P"]):
        if l == 0:
            fine = fine_nodes_level0(pr["xyz"], pr["cell_vtx"], p)
        else:
            fine = box_nodes(h["lo"][l], h["hi"][l], p)
        coarse = box_nodes(h["lo"][l + 1], h["hi"][l + 1], p)
        one = np.ones(P.shape[1])
        assert np.allclose(P @ one, 1.0, atol=1e-13)
        for _ in range(3):
            e = rng.integers(0, p + 1, size=d)
            f = lambda x: np.prod(x ** e[None, None, :], axis=2)
            # a global polynomial of degree <= p per variable restricted to
            # each agglomerate lies in Q_p(B_K): P maps it exactly
            assert np.allclose(P @ f(coarse).ravel(), f(fine).ravel(), atol=1e-12)


@pytest.mark.parametrize("name,n", [("c2", 16), ("c3", 4)])
def test_galerkin_symmetric_kernel(name, n):
    pr = make_problem(name, n=n)
    h = build_hierarchy(pr)
    A0, M, A, cM = system_matrix(pr)
    Al = A
    for P in h["P"]:
        Al = galerkin(Al, P)
        assert abs(Al - Al.T).max() <= 1e-14 * abs(Al).max()
        assert np.abs(Al @ np.ones(Al.shape[0])).max() < 1e-14 * abs(Al).max()


def _small_A0(name="c2", n=8):
    pr = make_problem(name, n=n)
    A0, M, A, cM = system_matrix(pr)
    return pr, A0


def test_lanczos_bounds_dense_eigenvalue():
    pr, A0 = _small_A0("c1", 8)
    d = A0.diagonal()
    S = (A0.toarray() / np.sqrt(d)[:, None]) / np.sqrt(d)[None, :]
    lam = np.linalg.eigvalsh(S)[-1]
    th = lanczos_theta_max(A0, d, 20)
    assert th <= lam * (1 + 1e-12)
    assert th >= 0.99 * lam
    # full Lanczos on a tiny matrix recovers the eigenvalue to roundoff
    pr2, A2 = _small_A0("c1", 2)
    d2 = A2.diagonal()
    S2 = (A2.toarray() / np.sqrt(d2)[:, None]) / np.sqrt(d2)[None, :]
    assert abs(lanczos_theta_max(A2, d2, 50) - np.linalg.eigvalsh(S2)[-1]) < 1e-10


def test_chebyshev_error_propagator_is_chebyshev_polynomial():
    pr, A0 = _small_A0("c1", 4)
    A = A0.toarray()
    d = np.diag(A)
    S = (A / np.sqrt(d)[:, None]) / np.sqrt(d)[None, :]
    lam, Q = np.linalg.eigh(S)
    lo, hi = 0.3 * lam[-1], 1.1 * lam[-1]
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    for k, s in ((3, 1), (3, 3), (2, 2), (1, 1)):
        T = np.polynomial.chebyshev.Chebyshev.basis(k)
        pk = T((theta - lam) / delta) / T(theta / delta)
        E = (Q * (pk ** s)[None, :]) @ Q.T
        E = (E / np.sqrt(d)[:, None]) * np.sqrt(d)[None, :]   # D^-1/2 E D^1/2
        x0 = np.random.default_rng(k).standard_normal(A.shape[0])
        x = chebyshev(A0, 1.0 / d, np.zeros_like(x0), x0, lo, hi, k, s)
        assert np.allclose(x, E @ x0, atol=1e-12 * np.abs(x0).max())


def _block_diag_dense(A, b):
    """The cells' diagonal blocks of A by dense slicing (independent of the
    oracle's sparse extraction)."""
    M = A.toarray()
    D = np.zeros_like(M)
    for K in range(M.shape[0] // b):
        s = slice(K * b, (K + 1) * b)
        D[s, s] = M[s, s]
    return D


def test_cell_block_inverse_and_lanczos_against_generalised_eigenvalues():
    """Cell-block Jacobi: D^-1 D = I per cell; the block Lanczos estimate
    bounds the largest generalised eigenvalue of (A, D) (scipy's symmetric
    generalised eigensolver) from below and recovers it with full Lanczos."""
    pr, A0 = _small_A0("c1", 8)
    b = 4
    D = _block_diag_dense(A0, b)
    Dk = diagonal_blocks(A0, b)
    for K in range(Dk.shape[0]):
        assert np.array_equal(Dk[K], D[K * b:(K + 1) * b, K * b:(K + 1) * b])
    Dinv = cell_block_inverse(A0, b).toarray()
    assert np.allclose(Dinv @ D, np.eye(D.shape[0]), atol=1e-12)
    assert np.abs(Dinv - Dinv.T).max() <= 1e-12 * np.abs(Dinv).max()
    lam = sla.eigh(A0.toarray(), D, eigvals_only=True)[-1]
    th = lanczos_theta_max_block(A0, b, 20)
    assert th <= lam * (1 + 1e-12) and th >= 0.99 * lam
    pr2, A2 = _small_A0("c1", 2)
    lam2 = sla.eigh(A2.toarray(), _block_diag_dense(A2, b), eigvals_only=True)[-1]
    assert abs(lanczos_theta_max_block(A2, b, 50) - lam2) < 1e-10
    # a block-diagonal operator is its own block Jacobi matrix: theta = 1
    from scipy.sparse import csr_matrix
    assert abs(lanczos_theta_max_block(csr_matrix(D), b, 20) - 1.0) < 1e-13


def test_chebyshev_cell_block_error_propagator():
    """With D the cells' diagonal blocks the smoother's error propagator is
    p(D^-1 A)^s, from the generalised eigenvectors A Q = D Q diag(lam),
    Q^T D Q = I, so that D^-1 A = Q diag(lam) Q^T D."""
    pr, A0 = _small_A0("c1", 4)
    b = 4
    A = A0.toarray()
    D = _block_diag_dense(A0, b)
    lam, Q = sla.eigh(A, D)
    lo, hi = 0.3 * lam[-1], 1.1 * lam[-1]
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    Dinv = cell_block_inverse(A0, b)
    for k, s in ((3, 1), (3, 3), (2, 2), (1, 1)):
        T = np.polynomial.chebyshev.Chebyshev.basis(k)
        pk = T((theta - lam) / delta) / T(theta / delta)
        E = (Q * (pk ** s)[None, :]) @ Q.T @ D
        x0 = np.random.default_rng(k).standard_normal(A.shape[0])
        x = chebyshev(A0, Dinv, np.zeros_like(x0), x0, lo, hi, k, s)
        assert np.allclose(x, E @ x0, atol=1e-12 * np.abs(x0).max())


def test_vcycle_cell_block_symmetric_positive():
    pr = make_problem("c2", n=8)
    h = build_hierarchy(pr)
    A0, M, A, cM = system_matrix(pr)
    mg = VCycle(A0, h["P"], jacobi="cell_block", b=9)
    B = _dense_op(mg, A0.shape[0])
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    with pytest.raises(ValueError):
        VCycle(A0, h["P"], jacobi="block")


def _dense_op(op, n):
    return np.stack([op(e) for e in np.eye(n)], axis=1)


def test_vcycle_symmetric_positive_and_special_cases():
    pr = make_problem("c2", n=8)
    h = build_hierarchy(pr)
    A0, M, A, cM = system_matrix(pr)
    mg = VCycle(A0, h["P"])
    B = _dense_op(mg, A0.shape[0])
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    # no smoothing: B = P A_c^-1 P^T on two levels
    pr2 = make_problem("c1", n=8)
    h2 = build_hierarchy(pr2)
    A02, _, _, _ = system_matrix(pr2)
    mg0 = VCycle(A02, h2["P"], sweeps=0)
    P = h2["P"][0].toarray()
    Ac = P.T @ A02.toarray() @ P
    assert np.allclose(_dense_op(mg0, A02.shape[0]), P @ np.linalg.solve(Ac, P.T),
                       atol=1e-12 * np.abs(np.linalg.inv(Ac)).max())
    # one level: B = A^-1
    mg1 = VCycle(A02, [])
    assert np.allclose(_dense_op(mg1, A02.shape[0]), np.linalg.inv(A02.toarray()),
                       rtol=1e-10, atol=1e-14)


def test_cholesky_coarse_factor():
    pr, A0 = _small_A0("c1", 4)
    A = A0.toarray()
    L = sla.cho_factor(A, lower=True)
    Lm = np.tril(L[0])
    assert np.allclose(Lm @ Lm.T, A, atol=1e-14 * np.abs(A).max())
    b = np.arange(A.shape[0], dtype=float)
    assert np.allclose(sla.cho_solve(L, b), np.linalg.solve(A, b), rtol=1e-12)


def test_pcg_against_dense_and_special_cases():
    pr = make_problem("c2", n=8)
    h = build_hierarchy(pr)
    A0, M, A, cM = system_matrix(pr)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A0.shape[0])
    xd = np.linalg.solve(A0.toarray(), b)
    mg = VCycle(A0, h["P"])
    x, st = pcg(A0, b, np.zeros_like(b), mg, 1e-13)
    assert st["converged"] and np.allclose(x, xd, rtol=0, atol=1e-11 * np.abs(xd).max())
    assert np.linalg.norm(b - A0 @ x) <= 2e-13 * st["r0"]
    # exact preconditioner: one iteration
    Ainv = np.linalg.inv(A0.toarray())
    x1, st1 = pcg(A0, b, np.zeros_like(b), lambda r: Ainv @ r, 1e-10)
    assert st1["its"] == 1
    # identity preconditioner: plain CG, converges within n iterations
    xi, sti = pcg(A0, b, np.zeros_like(b), lambda r: r, 1e-12, max_it=A0.shape[0])
    assert sti["converged"] and np.allclose(xi, xd, atol=1e-9 * np.abs(xd).max())
    # flexible beta agrees with the standard one for a fixed SPD preconditioner
    xf, stf = pcg(A0, b, np.zeros_like(b), mg, 1e-13, flexible=True)
    assert np.allclose(xf, xd, atol=1e-11 * np.abs(xd).max())
    # warm start equal to the solution: zero iterations
    x2, st2 = pcg(A0, A0 @ xd, xd, mg, 1e-10)
    assert st2["its"] <= 1


def test_str_packing_groups_and_nesting():
    """STR packing: a disjoint cover, groups of at most M with all but the
    tail of each strip full, nested levels, spatially compact groups."""
    from workloads.meshes import shell_mesh
    from oracle.hierarchy import str_partitions, str_pack
    xyz, cells, _ = shell_mesh(0.08)
    pars = str_partitions(xyz, cells, 8, 4)
    n = cells.shape[0]
    for par in pars:
        sizes = np.bincount(par)
        assert sizes.min() >= 1 and sizes.max() <= 8
        assert np.array_equal(np.unique(par), np.arange(len(sizes)))
        assert (sizes == 8).mean() > 0.9
        n = len(sizes)
    # compactness: group extent comparable to the fanout's cube root x h
    cen = xyz[cells].mean(axis=1)
    ext = np.zeros((len(np.unique(pars[0])), 3))
    for k in range(3):
        mx = np.full(ext.shape[0], -np.inf); mn = np.full(ext.shape[0], np.inf)
        np.maximum.at(mx, pars[0], cen[:, k]); np.minimum.at(mn, pars[0], cen[:, k])
        ext[:, k] = mx - mn
    assert np.median(ext.max(axis=1)) <= 3 * 0.08
    # 2D packing of a regular grid gives M-runs along y inside x-slabs
    c2 = np.stack(np.meshgrid(np.arange(8.0), np.arange(8.0), indexing="ij"), -1).reshape(-1, 2)
    par = str_pack(c2, 4)
    assert np.bincount(par).tolist() == [4] * 16
