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
    """Gauss-Lobatto points on [0, 1] for degree p <= 3 (interpolation nodes
    used to place initial values; p <= 2 coincides with equispaced)."""
    if p == 1:
        return np.array([0.0, 1.0])
    if p == 2:
        return np.array([0.0, 0.5, 1.0])
    if p == 3:
        s = np.sqrt(1.0 / 5.0)
        return np.array([0.0, 0.5 * (1.0 - s), 0.5 * (1.0 + s), 1.0])
    raise ValueError("p must be 1, 2 or 3")


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
