"""Mesh generators (inputs only).

Conventions shared by every consumer of these arrays:

* ``xyz``      float64 [n_vert, d]   vertex coordinates.
* ``cell_vtx`` int64   [n_cells, 2**d] corner vertex ids of each cell in
  lexicographic order (x fastest, then y, then z), i.e. corner
  ``c = c0 + 2*c1 + 4*c2`` sits at reference point ``(c0, c1, c2)``.
* Every cell is oriented the same way (its local x/y/z axes point along the
  global ones), so two face-neighbours see their shared face with the same
  tangential orientation.
"""
import numpy as np


def gl_nodes_1d(p):
    """Gauss-Lobatto points on [0, 1] for degree p <= 4 (interpolation nodes
    used to place initial values; p <= 2 coincides with equispaced)."""
    if p == 1:
        return np.array([0.0, 1.0])
    if p == 2:
        return np.array([0.0, 0.5, 1.0])
    if p == 3:
        s = np.sqrt(1.0 / 5.0)
        return np.array([0.0, 0.5 * (1.0 - s), 0.5 * (1.0 + s), 1.0])
    if p == 4:
        s = np.sqrt(3.0 / 7.0)
        return np.array([0.0, 0.5 * (1.0 - s), 0.5, 0.5 * (1.0 + s), 1.0])
    raise ValueError("p must be 1 to 4")


def structured_mesh(dim, n, jitter=0.0, seed=None, lo=0.0, hi=1.0):
    """Uniform n^dim grid of [lo, hi]^dim with optional seeded nodal jitter.

    Each vertex coordinate k is displaced by an independent draw from
    U(-jitter*h, +jitter*h) (numpy PCG64 stream of ``seed``), except that a
    coordinate stays fixed when the vertex lies on a boundary plane normal to
    axis k: boundary vertices slide tangentially, corners never move.
    """
    h = (hi - lo) / n
    ax = lo + h * np.arange(n + 1, dtype=np.float64)
    if dim == 2:
        X, Y = np.meshgrid(ax, ax, indexing="xy")          # X[j, i]
        xyz = np.stack([X.ravel(), Y.ravel()], axis=1)     # vertex i + (n+1) j
        I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
        idx = np.stack([I.ravel(), J.ravel()], axis=1)
    elif dim == 3:
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")   # [k, j, i]
        xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        K, J, I = np.meshgrid(np.arange(n + 1), np.arange(n + 1),
                              np.arange(n + 1), indexing="ij")
        idx = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    else:
        raise ValueError("dim must be 2 or 3")
    if jitter:
        rng = np.random.default_rng(seed)
        delta = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        movable = (idx > 0) & (idx < n)
        xyz = xyz + np.where(movable, delta, 0.0)
    nv = n + 1
    if dim == 2:
        j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        i = i.ravel(); j = j.ravel()                       # cell i + n j
        v0 = i + nv * j
        cells = np.stack([v0, v0 + 1, v0 + nv, v0 + nv + 1], axis=1)
    else:
        k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                              indexing="ij")
        i = i.ravel(); j = j.ravel(); k = k.ravel()        # cell i + n j + n^2 k
        v0 = i + nv * j + nv * nv * k
        s = nv * nv
        cells = np.stack([v0, v0 + 1, v0 + nv, v0 + nv + 1,
                          v0 + s, v0 + s + 1, v0 + s + nv, v0 + s + nv + 1],
                         axis=1)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(cells.astype(np.int64))


def cell_centroids(xyz, cell_vtx):
    """Vertex average of each cell."""
    return xyz[cell_vtx].mean(axis=1)


def dof_nodes(xyz, cell_vtx, p):
    """Physical positions of the DoF nodes, [n_cells, (p+1)^d, d].

    Node ``i = i0 + (p+1) i1 + (p+1)^2 i2`` of a cell sits at the multilinear
    image of the Gauss-Lobatto reference point ``(t[i0], t[i1], t[i2])``.
    Used only to sample initial values at nodes.
    """
    d = xyz.shape[1]
    t = gl_nodes_1d(p)
    q = p + 1
    if d == 2:
        ref = np.array([(t[a], t[b]) for b in range(q) for a in range(q)])
    else:
        ref = np.array([(t[a], t[b], t[c]) for c in range(q) for b in range(q)
                        for a in range(q)])
    # multilinear corner weights at each reference point
    w = np.ones((ref.shape[0], 2 ** d))
    for corner in range(2 ** d):
        for k in range(d):
            bit = (corner >> k) & 1
            w[:, corner] *= ref[:, k] if bit else (1.0 - ref[:, k])
    X = xyz[cell_vtx]                     # [n_cells, 2^d, d]
    return np.einsum("nc,kcd->knd", w, X)


def shell_mesh(h, outer=(1.0, 1.0, 2.5), inner=(0.7, 0.7, 2.0), z_base=0.0,
               jitter=0.15, seed=2603):
    """Voxel hexahedral mesh of a truncated thick ellipsoidal shell.

    Cells of a uniform grid of spacing h whose centres lie inside the outer
    ellipsoid (semi-axes ``outer``), outside the inner one and below the base
    plane z = z_base.  Vertices on the mesh surface stay fixed; every other
    vertex coordinate is displaced by U(-jitter*h, jitter*h) (PCG64 ``seed``).
    Cells keep the grid orientation (lexicographic corners).
    """
    ax, ay, az = outer
    lo = np.array([-ax, -ay, -az])
    n = np.ceil(np.array([2 * ax, 2 * ay, az + z_base]) / h).astype(int)
    I, J, K = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    c = lo + (np.stack([I, J, K], axis=-1) + 0.5) * h
    eo = (c[..., 0] / ax) ** 2 + (c[..., 1] / ay) ** 2 + (c[..., 2] / az) ** 2
    ei = (c[..., 0] / inner[0]) ** 2 + (c[..., 1] / inner[1]) ** 2 + (c[..., 2] / inner[2]) ** 2
    sel = (eo <= 1.0) & (ei > 1.0) & (c[..., 2] <= z_base)
    # cells in k-major, then j, then i order (x fastest)
    sel_t = np.transpose(sel, (2, 1, 0))
    kk, jj, ii = np.nonzero(sel_t)
    nv = n + 1
    def vid(i, j, k):
        return i + nv[0] * (j + nv[1] * k)
    corners = np.stack([vid(ii + (c_ & 1), jj + ((c_ >> 1) & 1), kk + ((c_ >> 2) & 1))
                        for c_ in range(8)], axis=1)
    uniq, inv = np.unique(corners.ravel(), return_inverse=True)
    cells = inv.reshape(-1, 8).astype(np.int64)
    vi = uniq % nv[0]
    vj = (uniq // nv[0]) % nv[1]
    vk = uniq // (nv[0] * nv[1])
    xyz = lo + np.stack([vi, vj, vk], axis=1) * h
    # surface vertices: those of faces without a selected neighbour
    pad = np.zeros(tuple(n + 2), dtype=bool)
    pad[1:-1, 1:-1, 1:-1] = sel
    on_surface = np.zeros(len(uniq), dtype=bool)
    face_corners = {(0, 0): [0, 2, 4, 6], (0, 1): [1, 3, 5, 7], (1, 0): [0, 1, 4, 5],
                    (1, 1): [2, 3, 6, 7], (2, 0): [0, 1, 2, 3], (2, 1): [4, 5, 6, 7]}
    for (axis, side), fcs in face_corners.items():
        off = [0, 0, 0]
        off[axis] = 1 if side else -1
        nb = pad[ii + 1 + off[0], jj + 1 + off[1], kk + 1 + off[2]]
        bnd = ~nb
        on_surface[cells[bnd][:, fcs].ravel()] = True
    rng = np.random.default_rng(seed)
    delta = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
    xyz = xyz + np.where(on_surface[:, None], 0.0, delta)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(cells), on_surface


def shell_transmural(points, outer=(1.0, 1.0, 2.5), inner=(0.7, 0.7, 2.0), iters=60):
    """Transmural coordinate t in [0, 1] (0 on the outer, 1 on the inner
    ellipsoid): the s for which the point lies on the ellipsoid with
    semi-axes (1-s) outer + s inner, by bisection."""
    o = np.asarray(outer)
    i_ = np.asarray(inner)
    lo = np.zeros(len(points))
    hi = np.ones(len(points))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        a = (1 - mid)[:, None] * o + mid[:, None] * i_
        f = ((points / a) ** 2).sum(axis=1) - 1.0
        # f < 0: inside the ellipsoid of parameter mid -> deeper than mid
        lo = np.where(f < 0, mid, lo)
        hi = np.where(f < 0, hi, mid)
    return np.clip(0.5 * (lo + hi), 0.0, 1.0)
