"""Evidence for the penalty reading on the jittered meshes (section 3: the
penalty coefficient defined right after the bilinear form a_h).

* 256x256 jittered Q2 square: with the paper's coefficient (factor 1) the
  assembled A_0 = c_M M + A has negative diagonal entries, so it is
  indefinite (e_i^T A_0 e_i < 0); with factor 2 it is positive definite,
  certified by the inertia of a symmetric factorisation.
* 1.0M-hex jittered shell: with the paper's coefficient the 16 x 16
  principal submatrix of A_0 on a pair of face-neighbour cells (located by
  tests/golden/make_c4_penalty_pair.py, which calls only the oracle) has a
  negative eigenvalue, so A_0 is indefinite; the shell takes factor 2 too.
* A coarser shell of the same construction (h = 0.06, 14,909 cells) is
  positive definite with the paper's coefficient: every face carries a
  positive definite share of A_0 (local certificate below).  The certificate
  is sufficient only.
"""
import json
import os
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from workloads import make_problem
from oracle.assemble import (assemble, cell_matrices, face_matrices, interior_faces,
                             system_matrix, unpack_sym)


def test_paper_penalty_is_indefinite_on_the_jittered_square():
    """Factor 1 on the seeded 256x256 mesh: some diagonal entries of A_0 are
    negative, a certificate of indefiniteness."""
    pr = make_problem("c2", penalty=("paper", 1.0))
    A0, _, _, _ = system_matrix(pr)
    d = A0.diagonal()
    assert (d < 0).sum() >= 1, d.min()
    assert d.min() < -1e-4


@pytest.mark.slow
def test_doubled_penalty_is_positive_definite_on_the_jittered_square():
    """Factor 2 (the configured value): Sylvester's law of inertia on a
    symmetric-mode factorisation without row pivoting.  A_0 = P^T L U P with
    the same permutation on rows and columns, so U's diagonal carries the
    inertia of A_0: no non-positive pivot means A_0 is positive definite."""
    pr = make_problem("c2")
    assert pr["penalty"] == ("paper", 2.0)
    A0, _, _, _ = system_matrix(pr)
    lu = sla.splu(A0.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                  options=dict(SymmetricMode=True))
    assert np.array_equal(lu.perm_r, lu.perm_c)
    piv = lu.U.diagonal()
    assert (piv <= 0).sum() == 0, piv.min()


def _face_share_certificate(pr):
    """Smallest eigenvalue over the faces of the local matrices
    B_F = A_F + sum_{K in F} (S_K + c_M M_K) / n_K, where A_F is the face's
    2b x 2b interior-penalty matrix and n_K the number of interior faces of
    K.  A_0 = sum_F B_F (every cell has a face), so all B_F >= 0 proves
    A_0 >= 0, and all B_F > 0 proves it positive definite."""
    xyz, cells, p = pr["xyz"], pr["cell_vtx"], pr["p"]
    d = xyz.shape[1]
    nc = cells.shape[0]
    X = xyz[cells]
    Dm = unpack_sym(pr["D_cell"], d)
    Mk, Sk, vol = cell_matrices(X, Dm, p)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    plus, minus, axis = interior_faces(cells, d)
    nK = np.bincount(plus, minlength=nc) + np.bincount(minus, minlength=nc)
    assert nK.min() >= 1
    share = (Sk + cM * Mk) / nK[:, None, None]
    b = Mk.shape[1]
    lmin = np.inf
    for k in range(d):
        sel = np.flatnonzero(axis == k)
        fp, fm = plus[sel], minus[sel]
        Bf = face_matrices(X[fp], X[fm], Dm[fp], Dm[fm], k, vol[fp], vol[fm], p, pr["penalty"])
        Bf[:, :b, :b] += share[fp]
        Bf[:, b:, b:] += share[fm]
        # relative to each block's own scale
        sc = np.abs(Bf).max(axis=(1, 2))
        lmin = min(lmin, (np.linalg.eigvalsh(Bf)[:, 0] / sc).min())
    return lmin


@pytest.mark.slow
def test_paper_penalty_is_indefinite_on_the_full_shell():
    """Factor 1 on the 1.0M-hex shell: the stored pair of neighbour cells has
    an indefinite principal submatrix of A_0 (rows of just those two cells
    assembled here)."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c4_penalty_pair.json")))
    pr = make_problem("c4", penalty=("paper", g["penalty_factor"]))
    cells = np.array(g["cells"])
    M, A = assemble(pr, row_cells=cells)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    A0 = (cM * M + A).tocsr()
    dofs = (cells[:, None] * pr["b"] + np.arange(pr["b"])).ravel()
    S = A0[dofs][:, dofs].toarray()
    assert abs(S - S.T).max() <= 1e-15 * abs(S).max()
    ev = np.linalg.eigvalsh(S)
    assert ev[0] < -1e-4 * abs(S).max(), ev[:3]
    assert abs(ev[0] / abs(S).max() - g["min_eigenvalue_over_max_entry"]) < 1e-9


def test_paper_penalty_is_positive_definite_on_a_coarser_shell():
    """The shell construction at h = 0.06 (jitter 0.15 h, fibre conductivity)
    with the paper's coefficient: every local face matrix is positive
    definite."""
    pr = make_problem("c4", h=0.06, penalty=("paper", 1.0))
    assert pr["n_cells"] > 10000
    assert _face_share_certificate(pr) > 0


def test_certificate_detects_a_missing_penalty():
    """The certificate is sufficient only, and at the configured time step the
    mass term carries much of it.  With a long step (small mass term) and the
    penalty switched off it fails clearly, so it does discriminate."""
    pr = make_problem("c4", h=0.09, penalty=("fixed", 0.0), dt=5.0)
    assert _face_share_certificate(pr) < -1.0
