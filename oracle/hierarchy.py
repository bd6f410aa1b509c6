"""Nested agglomerated hierarchy, bounding boxes and prolongation matrices
(section 4, agglomeration procedure; section 5.1: nested spaces, Q_p on the
bounding box of each agglomerate, prolongation as the natural embedding).

Readings:
* on a structured mesh the R-tree levels are a structured hierarchy of
  coarser grids (section 6, two-dimensional test); the grid method here bins
  cell centroids (vertex averages) into a uniform grid of the mesh's
  bounding box, coarsened by an integer factor per level;
* the coarse basis of agglomerate K is the tensor Lagrange basis on
  Gauss-Lobatto nodes of its bounding box B_K (minimum bounding box of all
  vertices of its fine cells);
* P[(e,i),(K,j)] = l^K_j(x_i^e): the coarse basis function evaluated at the
  physical position of fine node i.  On axis-aligned cells and on every
  level >= 1 this is the exact embedding; on jittered cells it is nodal
  interpolation.

* on unstructured meshes an STR (sort-tile-recursive) bulk-loaded R-tree of
  fanout 8 stands in for the R*-tree; the agglomerates of level l are the
  leaves below the tree nodes l levels above the leaves.

Pins (tests/test_oracle_mg.py): partition is a disjoint cover and nests,
P 1_c = 1_f, P reproduces coarse polynomials at fine nodes; STR groups are
full (all but a few per strip hold exactly M items) and spatially compact.
"""
import numpy as np
import scipy.sparse as sp

from .basis import gl_nodes, lagrange_1d, multi_index, corner_shape


def grid_partitions(xyz, cells, n_cells_axis, factors):
    """Per-level parent arrays for grid grouping.

    Returns ``parents`` with parents[l][e] = id at level l+1 of entity e at
    level l.  Level-l agglomerate ids are the linear bin index (x fastest)
    on a grid of n_cells_axis / prod(factors[:l]) bins per axis.
    """
    d = xyz.shape[1]
    cen = xyz[cells].mean(axis=1)
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    fine_of = np.arange(cells.shape[0])   # a representative fine cell per entity
    parents = []
    nb = n_cells_axis
    for g in factors:
        nb = nb // g
        t = (cen - lo) / (hi - lo) * nb
        bins = np.clip(np.floor(t).astype(np.int64), 0, nb - 1)
        lin = np.zeros(cells.shape[0], dtype=np.int64)
        for k in reversed(range(d)):
            lin = lin * nb + bins[:, k]
        # level-(l+1) id of each fine cell, then of each level-l entity
        par = lin[fine_of]
        parents.append(par)
        # representative fine cell of each new agglomerate
        n_new = nb ** d
        rep = np.full(n_new, -1, dtype=np.int64)
        rep[lin[::-1]] = np.arange(cells.shape[0])[::-1]
        if np.any(rep < 0):
            raise ValueError("empty agglomerate")
        fine_of = rep
    return parents


def members_level0(parents, n_fine):
    """For each level l, the level-l id of every fine cell."""
    ids = [np.arange(n_fine)]
    for par in parents:
        ids.append(par[ids[-1]])
    return ids


def bounding_boxes(xyz, cells, fine_ids, n_agg):
    """Minimum bounding boxes (lo [n,d], hi [n,d]) of agglomerates."""
    d = xyz.shape[1]
    lo = np.full((n_agg, d), np.inf)
    hi = np.full((n_agg, d), -np.inf)
    cmin = xyz[cells].min(axis=1)
    cmax = xyz[cells].max(axis=1)
    np.minimum.at(lo, fine_ids, cmin)
    np.maximum.at(hi, fine_ids, cmax)
    return lo, hi


def fine_nodes_level0(xyz, cells, p):
    """Physical DoF nodes of the fine cells: multilinear image of the GL
    reference nodes, [nc, b, d]."""
    d = xyz.shape[1]
    t = gl_nodes(p)
    mi = multi_index(p, d)
    ref = t[mi]                                   # [b, d]
    psi, _ = corner_shape(d, ref)
    return np.einsum("ic,ncd->nid", psi, xyz[cells])


def box_nodes(lo, hi, p):
    """GL nodes of boxes, [n, b, d]."""
    d = lo.shape[1]
    t = gl_nodes(p)
    ref = t[multi_index(p, d)]
    return lo[:, None, :] + ref[None, :, :] * (hi - lo)[:, None, :]


def prolongation(fine_pts, parent, lo, hi, p):
    """CSR prolongation from level l+1 (boxes lo/hi) to level l whose
    entities have DoF points fine_pts [n_l, b, d]."""
    n_l, b, d = fine_pts.shape
    n_c = lo.shape[0]
    nodes = gl_nodes(p)
    mi = multi_index(p, d)
    a = lo[parent]                                  # [n_l, d]
    w = hi[parent] - a
    ref = (fine_pts - a[:, None, :]) / w[:, None, :]   # [n_l, b, d]
    val = np.ones((n_l, b, b))
    for k in range(d):
        lk, _ = lagrange_1d(nodes, ref[:, :, k].ravel())
        lk = lk.reshape(n_l, b, p + 1)
        val *= lk[:, :, mi[:, k]]                    # [n_l, i, j]
    rows = (np.arange(n_l)[:, None, None] * b + np.arange(b)[None, :, None])
    cols = (parent[:, None, None] * b + np.arange(b)[None, None, :])
    R = np.broadcast_to(rows, val.shape).ravel()
    C = np.broadcast_to(cols, val.shape).ravel()
    return sp.csr_matrix((val.ravel(), (R, C)), shape=(n_l * b, n_c * b))


def build_hierarchy(prob):
    """Parents, boxes and prolongations of the agglomerated hierarchy of a
    problem dict (grid grouping, or an STR-packed R-tree when the problem
    asks for one).  Returns dict(parents, lo, hi, P, n) with P[l] mapping
    level l+1 to level l."""
    xyz, cells, p = prob["xyz"], prob["cell_vtx"], prob["p"]
    if prob.get("agglo", ("grid",))[0] == "rtree_str":
        _, fanout, n_levels = prob["agglo"]
        parents = str_partitions(xyz, cells, fanout, n_levels)
    else:
        parents = grid_partitions(xyz, cells, prob["n"], prob["group"])
    ids = members_level0(parents, cells.shape[0])
    ns = [cells.shape[0]] + [int(i.max()) + 1 for i in ids[1:]]
    los, his = [None], [None]
    for l in range(1, len(ids)):
        lo, hi = bounding_boxes(xyz, cells, ids[l], ns[l])
        los.append(lo); his.append(hi)
    P = []
    for l in range(len(parents)):
        if l == 0:
            pts = fine_nodes_level0(xyz, cells, p)
        else:
            pts = box_nodes(los[l], his[l], p)
        P.append(prolongation(pts, parents[l], los[l + 1], his[l + 1], p))
    return dict(parents=parents, lo=los, hi=his, P=P, n=ns, ids=ids)


def str_pack(centers, M):
    """Sort-tile-recursive packing of items (centres [N, d]) into groups of
    at most M: sort by x into S^(d-1)*M-item slabs (S = smallest integer with
    S^d >= ceil(N/M)), each slab by y into S*M-item strips (3D), each strip by
    z, then consecutive runs of M.  Ties are broken by item id.  Returns the
    group id of every item (groups numbered in packing order)."""
    N, d = centers.shape
    P = -(-N // M)
    S = 1
    while S ** d < P:
        S += 1
    ids = np.arange(N)
    order = np.lexsort((ids, centers[:, 0]))
    parent = np.empty(N, dtype=np.int64)
    g = 0
    slab = S ** (d - 1) * M
    for a in range(0, N, slab):
        sl = order[a:a + slab]
        sl = sl[np.lexsort((sl, centers[sl, 1]))]
        runs = [sl]
        if d == 3:
            strip = S * M
            runs = []
            for b in range(0, len(sl), strip):
                st = sl[b:b + strip]
                runs.append(st[np.lexsort((st, centers[st, 2]))])
        for run in runs:
            for c in range(0, len(run), M):
                parent[run[c:c + M]] = g
                g += 1
    return parent


def str_partitions(xyz, cells, fanout, n_levels):
    """Nested agglomerates from an STR-packed R-tree: level l+1 packs the
    minimum bounding boxes of level l (leaves: the cells' boxes), and every
    tree node gathers the leaves below it (Algorithms 1 and 2)."""
    lo = xyz[cells].min(axis=1)
    hi = xyz[cells].max(axis=1)
    parents = []
    for _ in range(n_levels - 1):
        centers = 0.5 * (lo + hi)
        par = str_pack(centers, fanout)
        n_new = int(par.max()) + 1
        nlo = np.full((n_new, lo.shape[1]), np.inf)
        nhi = np.full((n_new, lo.shape[1]), -np.inf)
        np.minimum.at(nlo, par, lo)
        np.maximum.at(nhi, par, hi)
        parents.append(par)
        lo, hi = nlo, nhi
    return parents
