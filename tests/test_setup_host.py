"""The library's host setup (assembly, agglomeration, prolongation, Galerkin
products, Lanczos) against the independent oracle, on the CPU."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2602_16312_amd import problem
from paper_2602_16312_amd import _ffi as F
from workloads import make_problem
from oracle.assemble import system_matrix
from oracle.hierarchy import build_hierarchy as oracle_hierarchy
from oracle.mg import VCycle


def dense_level(ex):
    d, fc, fb = ex["diag"], ex["face_cells"], ex["face_blocks"]
    n, b, _ = d.shape
    rows, cols, vals = [], [], []
    loc = np.arange(b)
    for K in range(n):
        rows.append(np.repeat(K * b + loc, b)); cols.append(np.tile(K * b + loc, b))
        vals.append(d[K].ravel())
    for f, (p, m) in enumerate(fc):
        rows.append(np.repeat(p * b + loc, b)); cols.append(np.tile(m * b + loc, b))
        vals.append(fb[f].ravel())
        rows.append(np.repeat(m * b + loc, b)); cols.append(np.tile(p * b + loc, b))
        vals.append(fb[f].T.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * b, n * b))


CASES = [("c1", 8, {}), ("c2", 16, {}), ("c2", 32, {"p": 1}), ("c3", 4, {}),
         ("c1", 8, {"bdf": 1}), ("c2", 8, {"p": 3, "group": [4]}), ("c2", 8, {"p": 4, "group": [4]})]


@pytest.mark.parametrize("name,n,kw", CASES)
def test_levels_match_oracle(name, n, kw):
    bdf = kw.pop("bdf", 2)
    pr = make_problem(name, n=n, **kw)
    h, s = problem.build(pr, device_setup=False, bdf=bdf)
    A0, M, A, cM = system_matrix(pr, bdf=bdf)
    oh = oracle_hierarchy(pr)
    mg = VCycle(A0, oh["P"])
    info = s.info()
    assert info["n_cells"] == oh["n"]
    for l in range(info["n_levels"]):
        ex = s.export_level(l)
        Al = dense_level(ex)
        ref = mg.A[l]
        assert abs(Al - ref).max() <= 1e-12 * abs(ref).max(), l
        if l + 1 < info["n_levels"]:
            assert np.array_equal(ex["parents"], oh["parents"][l])
            b = info["b"]
            Pl = oh["P"][l].toarray()
            for e in range(0, ex["P"].shape[0], max(1, ex["P"].shape[0] // 7)):
                K = ex["parents"][e]
                assert np.allclose(ex["P"][e], Pl[e * b:(e + 1) * b, K * b:(K + 1) * b],
                                   atol=1e-13)
    for l in range(info["n_levels"] - 1):
        assert abs(info["lam_hi"][l] - mg.lam[l][1]) <= 1e-10 * mg.lam[l][1]
        assert abs(info["lam_lo"][l] - mg.lam[l][0]) <= 1e-10 * mg.lam[l][0]


def test_cell_scaling_and_fixed_penalty():
    pr = make_problem("c1", n=8)
    rng = np.random.default_rng(11)
    s_cell = rng.uniform(0.5, 2.0, pr["n_cells"])
    h, s = problem.build(pr, device_setup=False, cell_scale=s_cell)
    A0, M, A, cM = system_matrix(pr, scale=s_cell)
    Al = dense_level(s.export_level(0))
    assert abs(Al - A0).max() <= 1e-12 * abs(A0).max()


def test_operator_complexity_and_counts():
    pr = make_problem("c2", n=64)
    h, s = problem.build(pr, device_setup=False)
    info = s.info()
    assert info["n_cells"] == [4096, 256, 16]
    assert info["n_dofs"] == 4096 * 9
    # 4x4 grouping on a grid: each coarse level has ~1/16 of the blocks
    assert 1.0 < info["op_complexity"] < 1.08


def test_str_hierarchy_and_shell_levels_match_oracle():
    """STR R-tree agglomeration (library C++ vs oracle numpy) is identical on
    the jittered shell, and the Galerkin levels built on it agree."""
    pr = make_problem("c4", h=0.09)
    h, s = problem.build(pr, device_setup=False)
    oh = oracle_hierarchy(pr)
    for l in range(len(oh["parents"])):
        assert np.array_equal(h.parents(l), oh["parents"][l])
    A0, M, A, cM = system_matrix(pr)
    mg = VCycle(A0, oh["P"])
    info = s.info()
    assert info["n_cells"] == oh["n"]
    for l in range(info["n_levels"]):
        Al = dense_level(s.export_level(l))
        assert abs(Al - mg.A[l]).max() <= 1e-12 * abs(mg.A[l]).max(), l
    assert 1.1 < info["op_complexity"] < 1.4


def test_paper_2d_test_dof_counts():
    """The paper's two-dimensional test (128x128 quadrilaterals, Q1-Q4) set up
    by the library has exactly the DoF counts of the paper's table dofs_2D."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_dof_counts.json")))
    table = g["fine_meshes"][0]
    assert table["cells"] == 128 * 128
    for p in (1, 2, 3, 4):
        pr = make_problem("e1", p=p)
        h, s = problem.build(pr, device_setup=False)
        assert s.info()["n_dofs"] == table["dofs"][str(p)]


def test_device_setup_option_needs_device_data():
    """The GPU set-up of the hierarchy is rejected without device set-up, and
    unknown set-up places are rejected by the binding."""
    from paper_2602_16312_amd._ffi import DGMGError
    pr = make_problem("c1", n=8)
    with pytest.raises(DGMGError):
        problem.build(pr, device_setup=False, setup="device")
    with pytest.raises(ValueError):
        problem.build(pr, device_setup=False, setup="gpu")


@pytest.mark.parametrize("name,kw", [("c2", dict(n=16)), ("c4", dict(h=0.09)), ("c3", dict(n=4))])
def test_hierarchy_boxes_match_oracle(name, kw):
    """The agglomerates' bounding boxes (the supports of the coarse bases) as
    exported by the library equal the oracle's (min/max are exact), and the
    level-0 boxes are the cells' own vertex ranges."""
    pr = make_problem(name, **kw)
    h, s = problem.build(pr, device_setup=False)
    oh = oracle_hierarchy(pr)
    d = pr["dim"]
    lo0, hi0 = h.boxes(0, d)
    X = pr["xyz"][pr["cell_vtx"]]
    assert np.array_equal(lo0, X.min(axis=1)) and np.array_equal(hi0, X.max(axis=1))
    for l in range(1, len(oh["n"])):
        lo, hi = h.boxes(l, d)
        assert np.array_equal(lo, oh["lo"][l]) and np.array_equal(hi, oh["hi"][l]), l
    with pytest.raises(F.DGMGError):
        h.boxes(len(oh["n"]), d)


@pytest.mark.parametrize("name,kw", [("c1", dict(n=8)), ("c2", dict(n=16)), ("c3", dict(n=4)),
                                     ("c4", dict(h=0.09)), ("c2", dict(n=8, p=3, group=[4]))])
def test_cell_block_jacobi_lanczos_matches_oracle(name, kw):
    """Cell-block Jacobi: the library's Lanczos estimates on L^-1 A_l L^-T
    (host Cholesky of every diagonal cell block) equal the oracle's block
    variant on every smoothed level, and are below the point variant's."""
    pr = make_problem(name, **kw)
    b = (pr["p"] + 1) ** pr["dim"]
    h, s = problem.build(pr, device_setup=False, jacobi="cell_block")
    h2, s2 = problem.build(pr, device_setup=False)
    A0 = system_matrix(pr)[0]
    mg = VCycle(A0, oracle_hierarchy(pr)["P"], jacobi="cell_block", b=b)
    info, ip = s.info(), s2.info()
    for l in range(info["n_levels"] - 1):
        assert abs(info["lam_hi"][l] - mg.lam[l][1]) <= 1e-10 * mg.lam[l][1], l
        assert abs(info["lam_lo"][l] - mg.lam[l][0]) <= 1e-10 * mg.lam[l][0], l
        assert info["lam_hi"][l] < ip["lam_hi"][l], l


def test_cell_block_jacobi_options():
    pr = make_problem("c1", n=8)
    with pytest.raises(ValueError):
        problem.build(pr, device_setup=False, jacobi="block")
    with pytest.raises(F.DGMGError):
        problem.build(pr, device_setup=False, jacobi="cell_block", max_rhs=8)
