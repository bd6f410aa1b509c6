"""SIPDG assembly of the mass matrix M and the diffusion matrix A as global
scalar CSR matrices (section 3: the forms a_h and m_h and the matrices of
eq. (matrices); penalty definition right after a_h).

Readings of the paper used here (listed in the design notes):
* the penalty term enters a_h with a plus sign (standard symmetric interior
  penalty); the printed form puts it under the minus, which is indefinite;
* on an interior face F between K+ and K-, alpha = c * p(p+1) *
  mean(|F|/|K+|, |F|/|K-|) and sigma = alpha * mean(n^T D+ n, n^T D- n),
  evaluated at every face quadrature point; c = 1 is the paper's value, a
  larger c is a safety factor for strongly distorted meshes; a fixed eta
  replaces alpha when requested;
* boundary faces contribute nothing (homogeneous Neumann);
* D is constant per cell (input), optionally scaled per cell by s_K; each
  side of a face uses its own scaled tensor;
* Gauss-Legendre rules with p+1 points per direction on cells and faces,
  multilinear (Q1) geometry.

Pins (tests/test_oracle_assembly.py, tests/test_oracle_geometry3d.py,
tests/test_oracle_penalty.py): 1^T M 1 = |Omega|, closed-form mass on boxes,
A 1 = 0, u^T A u = c^T D c |Omega| for linear u, v^T A u = int D grad u .
grad v for continuous polynomials, symmetry, positive spectrum of c_M M + A,
manufactured-solution convergence rates in 2D and on jittered hexahedra; on
curved hexahedral faces the consistency term against exact vector areas of
bilinear faces and the penalty term against tangent-cross-product normals
and area elements; the indefiniteness of the paper's penalty on the seeded
jittered square (and the inertia of the doubled one).
"""
import numpy as np
import scipy.sparse as sp

from .basis import tensor_basis, tensor_rule, cell_geometry


def unpack_sym(Dp, d):
    """Packed symmetric tensors (xx,xy,yy) / (xx,xy,xz,yy,yz,zz) -> [n,d,d]."""
    n = Dp.shape[0]
    D = np.zeros((n, d, d))
    if d == 2:
        D[:, 0, 0], D[:, 0, 1], D[:, 1, 1] = Dp[:, 0], Dp[:, 1], Dp[:, 2]
        D[:, 1, 0] = D[:, 0, 1]
    else:
        D[:, 0, 0], D[:, 0, 1], D[:, 0, 2] = Dp[:, 0], Dp[:, 1], Dp[:, 2]
        D[:, 1, 1], D[:, 1, 2], D[:, 2, 2] = Dp[:, 3], Dp[:, 4], Dp[:, 5]
        D[:, 1, 0], D[:, 2, 0], D[:, 2, 1] = D[:, 0, 1], D[:, 0, 2], D[:, 1, 2]
    return D


def face_corners(d, k, side):
    """Corners of the reference face xi_k = side, in increasing corner id."""
    return [c for c in range(2 ** d) if ((c >> k) & 1) == side]


def interior_faces(cell_vtx, d):
    """Interior faces as arrays (plus_cell, minus_cell, axis).

    A face is shared by exactly two cells; the plus cell sees it at
    xi_axis = 1 and the minus cell at xi_axis = 0, with identical tangential
    orientation (checked; anything else raises).
    """
    nc = cell_vtx.shape[0]
    recs = []
    for k in range(d):
        for side in (0, 1):
            fv = cell_vtx[:, face_corners(d, k, side)]
            recs.append((k, side, fv))
    allv = np.concatenate([np.sort(r[2], axis=1) for r in recs], axis=0)
    owner = np.concatenate([np.arange(nc)] * (2 * d))
    ax = np.concatenate([np.full(nc, r[0]) for r in recs])
    sd = np.concatenate([np.full(nc, r[1]) for r in recs])
    ordered = np.concatenate([r[2] for r in recs], axis=0)
    _, inv, cnt = np.unique(allv, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if cnt.max() > 2:
        raise ValueError("non-manifold face")
    order = np.argsort(inv, kind="stable")
    g = inv[order]
    first = np.flatnonzero(np.r_[True, g[1:] != g[:-1]])
    pairs = [(order[i], order[i + 1]) for i in first if cnt[g[i]] == 2]
    plus, minus, axis = [], [], []
    for a, b in pairs:
        if sd[a] == 0:
            a, b = b, a
        if ax[a] != ax[b] or sd[a] != 1 or sd[b] != 0:
            raise ValueError("inconsistently oriented neighbours")
        if not np.array_equal(ordered[a], ordered[b]):
            raise ValueError("face vertex order mismatch")
        plus.append(owner[a]); minus.append(owner[b]); axis.append(ax[a])
    return (np.array(plus, dtype=np.int64), np.array(minus, dtype=np.int64),
            np.array(axis, dtype=np.int64))


def cell_matrices(X, Dmat, p):
    """Per-cell mass and stiffness matrices and cell volumes.

    M_K[i,j] = sum_q w_q |det J| phi_i phi_j
    S_K[i,j] = sum_q w_q |det J| (J^-T grad phi_i)^T D_K (J^-T grad phi_j)
    """
    d = X.shape[2]
    xi, w = tensor_rule(p + 1, d)
    phi, gref = tensor_basis(p, d, xi)
    _, _, detJ, JinvT = cell_geometry(X, xi)
    if np.any(detJ <= 0):
        raise ValueError("non-positive Jacobian")
    wd = w[None, :] * np.abs(detJ)                       # [nc, nq]
    Mk = np.einsum("nq,qi,qj->nij", wd, phi, phi)
    G = np.einsum("nqab,qib->nqia", JinvT, gref)          # physical grads
    DG = np.einsum("nab,nqib->nqia", Dmat, G)
    Sk = np.einsum("nq,nqia,nqja->nij", wd, G, DG)
    vol = wd.sum(axis=1)
    return Mk, Sk, vol


def face_matrices(Xp, Xm, Dp, Dm, axis, volp, volm, p, penalty):
    """Local 2b x 2b matrices of the interior-face part of a_h for a batch of
    faces that all share the same reference axis.

    Unknown ordering within a local matrix: the b DoFs of K+ then those of K-.
    a_F(u, v) = - int {D grad u}.n [v] - int {D grad v}.n [u]
                + int sigma [u][v],
    with n the unit normal out of K+ and [v] = v+ - v-.
    """
    d = Xp.shape[2]
    tang = [m for m in range(d) if m != axis]
    ft, fw = tensor_rule(p + 1, d - 1)
    nq = ft.shape[0]
    xip = np.zeros((nq, d)); xim = np.zeros((nq, d))
    xip[:, axis] = 1.0
    xim[:, axis] = 0.0
    for j, m in enumerate(tang):
        xip[:, m] = ft[:, j]
        xim[:, m] = ft[:, j]
    phip, grp = tensor_basis(p, d, xip)
    phim, grm = tensor_basis(p, d, xim)
    xp_, _, detp, JiTp = cell_geometry(Xp, xip)
    xm_, _, detm, JiTm = cell_geometry(Xm, xim)
    # Nanson: n dS = det J J^-T e_axis dS_ref (for K+, outward is +e_axis)
    nvec = JiTp[:, :, :, axis]                            # [nf, nq, d]
    nrm = np.linalg.norm(nvec, axis=2)
    n = nvec / nrm[:, :, None]
    dS = np.abs(detp) * nrm * fw[None, :]                 # [nf, nq]
    area = dS.sum(axis=1)
    Gp = np.einsum("fqab,qib->fqia", JiTp, grp)
    Gm = np.einsum("fqab,qib->fqia", JiTm, grm)
    fluxp = np.einsum("fqia,fab,fqb->fqi", Gp, Dp, n)     # (D+ grad phi+).n
    fluxm = np.einsum("fqia,fab,fqb->fqi", Gm, Dm, n)
    nDn = 0.5 * (np.einsum("fqa,fab,fqb->fq", n, Dp, n)
                 + np.einsum("fqa,fab,fqb->fq", n, Dm, n))
    if penalty[0] == "paper":
        c = float(penalty[1]) if len(penalty) > 1 else 1.0
        eta = c * p * (p + 1) * 0.5 * (area / volp + area / volm)
    else:
        eta = np.full(Xp.shape[0], float(penalty[1]))
    sig = eta[:, None] * nDn                              # [nf, nq]
    nf = Xp.shape[0]
    b = phip.shape[1]
    jump = np.concatenate([np.broadcast_to(phip, (nf, nq, b)),
                           -np.broadcast_to(phim, (nf, nq, b))], axis=2)
    flux = np.concatenate([fluxp, fluxm], axis=2)         # D grad phi . n
    T1 = -0.5 * np.einsum("fq,fqI,fqJ->fIJ", dS, jump, flux)   # -{D grad u}.n [v]
    T3 = np.einsum("fq,fqI,fqJ->fIJ", dS * sig, jump, jump)
    return T1 + T1.transpose(0, 2, 1) + T3


def assemble(prob, scale=None, row_cells=None):
    """Global CSR matrices (M, A) for a problem dict from ``workloads``.

    ``scale`` multiplies D_K per cell (default 1).  ``row_cells`` restricts
    the assembled rows to the DoFs of those cells (all columns kept), for
    sampled checks on meshes too large to assemble whole.
    """
    xyz, cells, p = prob["xyz"], prob["cell_vtx"], prob["p"]
    d = xyz.shape[1]
    nc = cells.shape[0]
    b = (p + 1) ** d
    N = nc * b
    Dmat = unpack_sym(prob["D_cell"], d)
    if scale is not None:
        Dmat = Dmat * np.asarray(scale)[:, None, None]
    X = xyz[cells]
    rowmask = np.ones(nc, dtype=bool)
    if row_cells is not None:
        rowmask[:] = False
        rowmask[np.asarray(row_cells)] = True
    plus, minus, axis = interior_faces(cells, d)
    keepf = rowmask[plus] | rowmask[minus]
    need = rowmask.copy()
    need[plus[keepf]] = True
    need[minus[keepf]] = True
    cid = np.flatnonzero(need)
    Mk, Sk, vol_sub = cell_matrices(X[cid], Dmat[cid], p)
    vol = np.zeros(nc)
    vol[cid] = vol_sub
    loc = np.arange(b)
    rows_m, cols_m, vals_m = [], [], []
    rows_a, cols_a, vals_a = [], [], []
    own = rowmask[cid]
    base = cid[own][:, None, None] * b
    rr = np.broadcast_to(base + loc[None, :, None], (own.sum(), b, b))
    cc = np.broadcast_to(base + loc[None, None, :], (own.sum(), b, b))
    rows_m.append(rr.ravel()); cols_m.append(cc.ravel()); vals_m.append(Mk[own].ravel())
    rows_a.append(rr.ravel()); cols_a.append(cc.ravel()); vals_a.append(Sk[own].ravel())
    for k in range(d):
        sel = np.flatnonzero(keepf & (axis == k))
        if sel.size == 0:
            continue
        fp, fm = plus[sel], minus[sel]
        Af = face_matrices(X[fp], X[fm], Dmat[fp], Dmat[fm], k, vol[fp],
                           vol[fm], p, prob["penalty"])
        dofs = np.concatenate([fp[:, None] * b + loc[None, :],
                               fm[:, None] * b + loc[None, :]], axis=1)
        R = np.broadcast_to(dofs[:, :, None], Af.shape)
        C = np.broadcast_to(dofs[:, None, :], Af.shape)
        rows_a.append(R.ravel()); cols_a.append(C.ravel()); vals_a.append(Af.ravel())
    rm = np.concatenate(rows_m); cm = np.concatenate(cols_m)
    ra = np.concatenate(rows_a); ca = np.concatenate(cols_a)
    va = np.concatenate(vals_a)
    if row_cells is not None:
        keep = rowmask[ra // b]
        ra, ca, va = ra[keep], ca[keep], va[keep]
    M = sp.csr_matrix((np.concatenate(vals_m), (rm, cm)), shape=(N, N))
    A = sp.csr_matrix((va, (ra, ca)), shape=(N, N))
    M.sum_duplicates(); A.sum_duplicates()
    return M, A


def mass_blocks(prob):
    """Per-cell mass blocks [n_cells, b, b] (used to form M f for nodal f)."""
    xyz, cells, p = prob["xyz"], prob["cell_vtx"], prob["p"]
    d = xyz.shape[1]
    Mk, _, _ = cell_matrices(xyz[cells], np.zeros((cells.shape[0], d, d)), p)
    return Mk


def system_matrix(prob, scale=None, bdf=2):
    """A_0 = c_M M + A with c_M = alpha_t chi C_m / dt; alpha_t = 3/2 for BDF2
    (eq. fully_discrete), 1 for backward Euler."""
    M, A = assemble(prob, scale)
    cM = (1.5 if bdf == 2 else 1.0) * prob["chi"] * prob["Cm"] / prob["dt"]
    return (cM * M + A).tocsr(), M, A, cM
