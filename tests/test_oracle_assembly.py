"""Pins of the oracle's SIPDG assembly (section 3, forms a_h and m_h).

Each check is fixed by mathematics outside the assembler: areas, closed-form
1D mass matrices, the kernel of the Neumann operator, energies of linear and
polynomial fields, symmetry/definiteness, and manufactured-solution rates."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workloads import make_problem
from workloads.meshes import structured_mesh
from oracle.assemble import assemble, interior_faces, mass_blocks, system_matrix, unpack_sym
from oracle.basis import multi_index, tensor_basis, tensor_rule, cell_geometry
from oracle.hierarchy import fine_nodes_level0

CASES = [("c1", 6), ("c2", 6), ("c3", 3)]


def _prob(name, n, **kw):
    return make_problem(name, n=n, **kw)


@pytest.mark.parametrize("name,n", CASES)
def test_mass_total_is_domain_measure(name, n):
    pr = _prob(name, n)
    M, _ = assemble(pr)
    one = np.ones(pr["N"])
    assert abs(one @ (M @ one) - 1.0) < 1e-13


def test_mass_block_closed_form_on_boxes():
    # 1D Lagrange mass matrices on [0,h] for GL nodes p = 1, 2 (closed form)
    m1 = np.array([[2, 1], [1, 2]]) / 6.0
    m2 = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0
    for p, m in ((1, m1), (2, m2)):
        pr = make_problem("c1", n=4, p=p)
        Mk = mass_blocks(pr)
        h = 0.25
        assert np.allclose(Mk[5], np.kron(m, m) * h * h, atol=1e-15)
    pr = make_problem("c3", n=2)
    Mk = mass_blocks(pr)
    assert np.allclose(Mk[3], np.kron(m2, np.kron(m2, m2)) * 0.5 ** 3, atol=1e-15)


@pytest.mark.parametrize("name,n", CASES)
def test_constants_in_kernel_and_symmetry(name, n):
    pr = _prob(name, n)
    _, A = assemble(pr)
    one = np.ones(pr["N"])
    assert np.abs(A @ one).max() < 1e-15 * 1e3
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()


@pytest.mark.parametrize("name,n", CASES)
def test_linear_field_energy(name, n):
    """u = c.x lies in the mapped space; jumps vanish, so
    u^T A u = c^T D c |Omega| and u^T M u = int (c.x)^2 exactly."""
    pr = _prob(name, n)
    d = pr["dim"]
    # use a constant tensor so the closed form is a single number
    D = np.array([1.3, 0.2, 0.7]) if d == 2 else np.array([1.1, 0.1, -0.2, 0.9, 0.05, 0.6])
    pr["D_cell"] = np.tile(D, (pr["n_cells"], 1))
    M, A = assemble(pr)
    x = fine_nodes_level0(pr["xyz"], pr["cell_vtx"], pr["p"]).reshape(-1, d)
    c = np.array([0.7, -1.2, 0.4][:d])
    u = x @ c
    Dm = unpack_sym(D[None], d)[0]
    assert abs(u @ (A @ u) - c @ Dm @ c) < 1e-12
    # int_[0,1]^d (c.x)^2 = sum c_k^2/3 + sum_{k!=m} c_k c_m / 4
    exact = (c ** 2).sum() / 3 + (c.sum() ** 2 - (c ** 2).sum()) / 4
    assert abs(u @ (M @ u) - exact) < 1e-13


def test_polynomial_bilinear_form_closed_form():
    """Continuous quadratics on an axis-aligned Q2 mesh: v^T A u equals
    int sigma grad u . grad v; u = x^2, v = x y gives sigma * 1/2."""
    pr = make_problem("c1", n=4, p=2)
    _, A = assemble(pr)
    x = fine_nodes_level0(pr["xyz"], pr["cell_vtx"], 2).reshape(-1, 2)
    u = x[:, 0] ** 2
    v = x[:, 0] * x[:, 1]
    assert abs(v @ (A @ u) - 1e-3 * 0.5) < 1e-16
    w = x[:, 1] ** 2
    # int grad(x^2).grad(y^2) = 0,  int |grad x^2|^2 = 4/3
    assert abs(w @ (A @ u)) < 1e-15
    assert abs(u @ (A @ u) - 1e-3 * 4.0 / 3.0) < 1e-15


@pytest.mark.parametrize("name,n", [("c1", 4), ("c2", 4), ("c3", 2)])
def test_spectrum(name, n):
    """A is symmetric positive semi-definite with exactly one zero mode
    (constants); c_M M + A is positive definite."""
    pr = _prob(name, n)
    A0, M, A, cM = system_matrix(pr)
    ev = np.linalg.eigvalsh(A.toarray())
    scale = ev[-1]
    assert abs(ev[0]) < 1e-12 * scale
    assert ev[1] > 1e-6 * scale
    assert np.linalg.eigvalsh(A0.toarray())[0] > 0


def test_wrong_penalty_sign_is_detected():
    """Planting the printed (minus) sign of the penalty in the oracle makes A
    indefinite, which the spectrum check above would catch."""
    import oracle.assemble as asm
    pr = make_problem("c2", n=4)
    orig = asm.face_matrices

    def flipped(*a, **k):
        full = orig(*a, **k)
        Xp, Xm, Dp, Dm, axis, volp, volm, p, pen = a
        # recompute the consistency part only and subtract the penalty twice
        nopen = orig(Xp, Xm, Dp, Dm, axis, volp, volm, p, ("fixed", 0.0))
        return nopen - (full - nopen)

    asm.face_matrices = flipped
    try:
        _, A = asm.assemble(pr)
    finally:
        asm.face_matrices = orig
    assert np.linalg.eigvalsh(A.toarray())[0] < -1e-8


def _l2_error(pr, U, fn):
    p, d = pr["p"], pr["dim"]
    xi, w = tensor_rule(p + 3, d)
    phi, _ = tensor_basis(p, d, xi)
    X = pr["xyz"][pr["cell_vtx"]]
    x, _, detJ, _ = cell_geometry(X, xi)
    uh = np.einsum("qi,ni->nq", phi, U.reshape(pr["n_cells"], -1))
    return np.sqrt((w[None] * np.abs(detJ) * (uh - fn(x)) ** 2).sum())


@pytest.mark.parametrize("p,jit", [(1, 0.0), (2, 0.0), (1, 0.2), (2, 0.2)])
def test_manufactured_solution_rates(p, jit):
    """(c M + A) u = M f with u = cos(pi x) cos(pi y), f = (c + 2 pi^2 s) u:
    L2 error decays at rate p+1 on structured and jittered meshes."""
    s, c = 1.0, 1.0
    errs = []
    ns = [8, 16, 32]
    for n in ns:
        pr = make_problem("c2", n=n, p=p, jitter=jit, sigma=("iso", s))
        M, A = assemble(pr)
        x = fine_nodes_level0(pr["xyz"], pr["cell_vtx"], p).reshape(-1, 2)
        fn = lambda y: np.cos(np.pi * y[..., 0]) * np.cos(np.pi * y[..., 1])
        f = (c + 2 * np.pi ** 2 * s) * fn(x)
        U = spla.spsolve((c * M + A).tocsc(), M @ f)
        errs.append(_l2_error(pr, U, fn))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.15, (rates, errs)


@pytest.mark.parametrize("name,kw", [("c1", dict(n=5)), ("c2", dict(n=5)), ("c2", dict(n=4, p=3)),
                                     ("c3", dict(n=3)), ("c3", dict(n=3, p=1))])
def test_face_blocks_vanish_off_the_face_nodes(name, kw):
    # Section 3: every face term of a_h has the trace of the test or of the
    # trial function as a factor, and a Lagrange function on Gauss-Lobatto
    # nodes has a zero trace on a face unless its node lies on that face.  So
    # the block A[plus, minus] of an interior face (plus sees it at xi_a = 1,
    # minus at xi_a = 0) is exactly zero outside the rows of plus's face nodes
    # and the columns of minus's face nodes; the rest carries the coupling.
    pr = _prob(name, **kw)
    _, A = assemble(pr)
    A = A.tocsr()
    d, p = pr["xyz"].shape[1], pr["p"]
    b = (p + 1) ** d
    mi = multi_index(p, d)
    plus, minus, axis = interior_faces(pr["cell_vtx"], d)
    assert len(plus) > 0
    for K, Nb, a in zip(plus, minus, axis):
        blk = A[K * b:(K + 1) * b, Nb * b:(Nb + 1) * b].toarray()
        allowed = (mi[:, a] == p)[:, None] | (mi[:, a] == 0)[None, :]
        assert np.all(blk[~allowed] == 0.0)
        assert np.count_nonzero(blk[allowed]) > 0.5 * allowed.sum()
