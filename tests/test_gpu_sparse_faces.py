"""Sparse face blocks of the nodal fine level (axis-ELL): on a Lagrange basis
on Gauss-Lobatto nodes, entry (i, j) of a face block vanishes unless node i
or node j lies on the face (section 3, face terms of a_h), and single-column
solvers store only the rest.  The level-0 products and a V-cycle must equal
those of the same solver with whole face blocks bit for bit (the left-out
entries are exact zeros, and both kernels accumulate in the same order),
and the level-0 product must equal the oracle's A_0."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from oracle.assemble import system_matrix
from oracle.hierarchy import build_hierarchy as oracle_hierarchy
from oracle.mg import VCycle

pytestmark = pytest.mark.gpu

CASES = [("c1", dict(n=16)), ("c2", dict(n=24)), ("c2", dict(n=20, p=4, group=[4])),
         ("c3", dict(n=6)), ("c3", dict(n=6, p=1, group=[3])), ("c4", dict(h=0.09))]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _solvers(pr, precision):
    A0 = system_matrix(pr)[0]
    mg = VCycle(A0, oracle_hierarchy(pr)["P"])
    out = []
    for layout in ("axis_ell", "axis_ell_dense"):
        h, s = problem.build(pr, precision=precision, lam_override=mg.lam, fine_layout=layout)
        out.append((h, s))
    return A0, out


@pytest.mark.parametrize("name,kw", CASES)
def test_sparse_faces_equal_whole_blocks(name, kw):
    pr = make_problem(name, **kw)
    A0, ((_, sp), (_, de)) = _solvers(pr, "mixed")
    assert sp.info()["sparse_faces"] and sp.info()["fine_layout"] == "axis_ell"
    assert not de.info()["sparse_faces"]
    N = pr["N"]
    rng = np.random.default_rng(7)
    x = rng.standard_normal(N)
    ys = torch.empty(N, dtype=torch.float64, device="cuda")
    yd = torch.empty(N, dtype=torch.float64, device="cuda")
    for prec in ("fp64", "mixed"):
        say("sparse faces apply", name, kw, prec)
        api.apply(sp, 0, dev(x), ys, prec)
        api.apply(de, 0, dev(x), yd, prec)
        assert np.array_equal(host(ys), host(yd)), prec
    assert rel(host(ys), A0 @ x) <= 2e-6
    api.apply(sp, 0, dev(x), ys, "fp64")
    assert rel(host(ys), A0 @ x) <= 1e-13
    say("sparse faces vcycle", name, kw)
    r = rng.standard_normal(N)
    api.vcycle(sp, dev(r), ys)
    api.vcycle(de, dev(r), yd)
    assert np.array_equal(host(ys), host(yd))


def test_multi_column_solvers_keep_whole_blocks():
    pr = make_problem("c2", n=24)
    h, s = problem.build(pr, precision="mixed", max_rhs=8)
    assert s.info()["fine_layout"] == "axis_ell" and not s.info()["sparse_faces"]


def test_fp64_solver_uses_sparse_faces():
    pr = make_problem("c2", n=24)
    A0 = system_matrix(pr)[0]
    h, s = problem.build(pr, precision="fp64", fine_layout="axis_ell")
    assert s.info()["sparse_faces"]
    x = np.random.default_rng(3).standard_normal(pr["N"])
    y = torch.empty(pr["N"], dtype=torch.float64, device="cuda")
    api.apply(s, 0, dev(x), y, "fp64")
    assert rel(host(y), A0 @ x) <= 1e-13
