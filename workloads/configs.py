"""The five benchmark/test problems, as plain input data.

Each ``make_problem(name)`` call returns a dict of numpy arrays and scalars.
Every value is either a constant stated by the problem definition or drawn
from a seeded numpy PCG64 stream; no solver arithmetic happens here.

Ionic parameter vectors (fixed order, shared by every consumer):

* FHN  ``[k, a, eps, gamma]``       (FitzHugh-Nagumo, section 2.2)
* AP   ``[k, a, eps0]``             (Aliev-Panfilov with mu1 = 0)
* BO   ``BO_PARAM_NAMES`` below      (Bueno-Orovio, section 2.2 and the
  appendix parameter table, time constants converted from s to ms)
"""
import numpy as np

from .meshes import (structured_mesh, cell_centroids, dof_nodes, shell_mesh,
                     shell_transmural)

BO_PARAM_NAMES = [
    "tau_o1", "tau_o2", "tau_so1", "tau_so2", "tau_si", "tau_fi",
    "tau_1p", "tau_1m1", "tau_1m2", "tau_2m1", "tau_2m2", "tau_3m1", "tau_3m2",
    "tau_2p", "tau_2inf", "k_2", "k_3", "k_so", "w_inf_star",
    "V_1", "V_1m", "V_2", "V_2m", "V_3", "V_hat", "V_o", "V_so", "u_o",
]

# Appendix table of Bueno-Orovio parameters.  Time constants are printed in
# seconds; the 3D workloads run in milliseconds, so every tau is multiplied by
# 1e3 except tau_2inf, which divides a potential and is dimensionless.  Rows
# duplicated in the printed table are taken once.  u_o = 0 makes the paper's
# initial state (u = 0, w = (1, 1, 0)) a rest state of the so-current.
BO_EPI = {
    "tau_o1": 6.0, "tau_o2": 6.0, "tau_so1": 43.0, "tau_so2": 0.2,
    "tau_si": 2.8723, "tau_fi": 0.11, "tau_1p": 1.4506, "tau_1m1": 60.0,
    "tau_1m2": 1150.0, "tau_2m1": 70.0, "tau_2m2": 20.0, "tau_3m1": 2.7342,
    "tau_3m2": 3.0, "tau_2p": 280.0, "tau_2inf": 0.07, "k_2": 65.0,
    "k_3": 2.0994, "k_so": 2.0, "w_inf_star": 0.94, "V_1": 0.3,
    "V_1m": 0.015, "V_2": 0.015, "V_2m": 0.03, "V_3": 0.9087, "V_hat": 1.58,
    "V_o": 0.006, "V_so": 0.65, "u_o": 0.0,
}

MODEL_IDS = {"fhn": 0, "ap": 1, "bo": 2}
N_GATES = {"fhn": 1, "ap": 1, "bo": 3}

CONFIGS = {
    # 32x32 Q1 unit square, FitzHugh-Nagumo, fixed penalty 10 p^2 / h
    "c1": dict(dim=2, n=32, p=1, jitter=0.0, seed=None, group=[4],
               sigma=("iso", 1e-3), chi=1.0, Cm=1.0, dt=1e-2, steps=10,
               model="fhn", params=[19.5, 0.13, 0.01, 0.5],
               penalty=("fixed", 10.0 * 1 ** 2 * 32), ic="corner_disc",
               stim=None, tol=1e-10),
    # 256x256 jittered Q2, Aliev-Panfilov, three levels (4x4 grouping twice).
    # The paper's penalty (factor 1) leaves A_0 indefinite on this seeded
    # mesh (negative diagonal entries at the most distorted cells); factor 2
    # makes it positive definite (no negative pivot in a symmetric
    # factorisation).
    "c2": dict(dim=2, n=256, p=2, jitter=0.2, seed=2602, group=[4, 4],
               sigma=("iso", 1e-3), chi=1.0, Cm=1.0, dt=1e-2, steps=100,
               model="ap", params=[8.0, 0.15, 0.002],
               penalty=("paper", 2.0), ic="corner_disc", stim=None, tol=1e-8),
    # 64^3 Q2 cube, rotating fibres, Bueno-Orovio (ms), four levels (2x2x2)
    "c3": dict(dim=3, n=64, p=2, jitter=0.0, seed=None, group=[2, 2, 2],
               sigma=("fibre_z", 1.2e-3, 2.5e-4), chi=1.0, Cm=1.0, dt=5e-2,
               steps=50, model="bo",
               params=[BO_EPI[k] for k in BO_PARAM_NAMES],
               penalty=("paper",), ic="rest", stim=("corner_block", 0.125, 0.3, 3.0),
               tol=1e-8),
    # ventricle-like truncated ellipsoidal shell (~1.0M voxel hexes, interior
    # nodes jittered +-0.15 h), Q1, transmural fibres, Bueno-Orovio (ms),
    # five STR R-tree levels of fanout 8, eight stimulus sites (apex + 7
    # endocardial) for the multi-right-hand-side runs.  The paper's penalty
    # (factor 1) leaves A_0 indefinite on this mesh: the 16 x 16 principal
    # submatrix of a pair of face-neighbour cells next to the surface has a
    # negative eigenvalue (and CG meets (p, A p) < 0); factor 2 as on the
    # jittered square.  On a coarser shell of the same construction
    # (h = 0.06) factor 1 is provably positive definite.
    "c4": dict(kind="shell", dim=3, h=0.0147, p=1, jitter=0.15, seed=2603,
               agglo=("rtree_str", 8, 5), group=[],
               sigma=("fibre_shell", 1.2e-3, 2.5e-4), chi=1.0, Cm=1.0, dt=5e-2,
               steps=20, model="bo", params=[BO_EPI[k] for k in BO_PARAM_NAMES],
               penalty=("paper", 2.0), ic="rest",
               stim=("sites", 0.15, 0.3, 3.0, 2604, 8), tol=1e-8),
    # the paper's two-dimensional test (section 6, first experiment): 128x128
    # unit square, FitzHugh-Nagumo with the appendix parameters (SI units),
    # electric shock on [0.4, 0.6]^2 for t <= 1 ms, T = 0.4 s, dt = 1e-4 s,
    # PCG stopped at absolute residual 1e-14; three grid-grouped levels
    # stand in for the unstated hierarchy
    "e1": dict(dim=2, n=128, p=1, jitter=0.0, seed=None, group=[4, 4],
               sigma=("iso", 0.12), chi=1e5, Cm=1e-2, dt=1e-4, steps=4000,
               model="fhn", params=[19.5, 0.013, 40.0, 0.1],
               penalty=("paper",), ic="rest", stim=("box", 0.4, 0.6, 2e6, 1e-3),
               tol=1e-14, tol_mode="abs"),
    # adjoint problem: mesh and physics of c2, 50 steps; the 64 sensors lie in
    # cells whose centroids are 0.08 to 0.16 from the stimulated corner, the
    # band the excitation front crosses within the 50 steps
    "c5": dict(dim=2, n=256, p=2, jitter=0.2, seed=2602, group=[4, 4],
               sigma=("iso", 1e-3), chi=1.0, Cm=1.0, dt=1e-2, steps=50,
               model="ap", params=[8.0, 0.15, 0.002],
               penalty=("paper", 2.0), ic="corner_disc", stim=None, tol=1e-8,
               sensors=(64, 2605, (0.08, 0.16)), target_seed=2606),
}


SHELL_OUTER = (1.0, 1.0, 2.5)
SHELL_INNER = (0.7, 0.7, 2.0)


def _shell_fibres(cen, sl, st):
    """D = st I + (sl - st) f f^T with f rotating from -60 deg (outer) to
    +60 deg (inner) with the transmural coordinate, in the plane spanned by
    the circumferential direction and the meridian tangent."""
    t = shell_transmural(cen, SHELL_OUTER, SHELL_INNER)
    th = np.deg2rad(-60.0 + 120.0 * t)
    r = np.hypot(cen[:, 0], cen[:, 1])
    ec = np.stack([-cen[:, 1], cen[:, 0], np.zeros(len(cen))], axis=1)
    ec = np.where(r[:, None] > 1e-12, ec / np.maximum(r, 1e-300)[:, None], np.array([1.0, 0.0, 0.0]))
    a = (1 - t)[:, None] * np.asarray(SHELL_OUTER) + t[:, None] * np.asarray(SHELL_INNER)
    nv = cen / a ** 2
    nv /= np.linalg.norm(nv, axis=1)[:, None]
    el = np.cross(nv, ec)
    el /= np.maximum(np.linalg.norm(el, axis=1), 1e-300)[:, None]
    f = np.cos(th)[:, None] * ec + np.sin(th)[:, None] * el
    D = st * np.eye(3)[None] + (sl - st) * f[:, :, None] * f[:, None, :]
    return np.stack([D[:, 0, 0], D[:, 0, 1], D[:, 0, 2], D[:, 1, 1], D[:, 1, 2], D[:, 2, 2]], axis=1)


def _stim_sites(nsites, seed):
    """Outer apex plus seeded endocardial points (inner ellipsoid, -1.8 < z < -0.3)."""
    rng = np.random.default_rng(seed)
    sites = [np.array([0.0, 0.0, -SHELL_OUTER[2]])]
    for _ in range(nsites - 1):
        z = rng.uniform(-1.8, -0.3)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        rr = np.sqrt(max(0.0, 1.0 - (z / SHELL_INNER[2]) ** 2))
        sites.append(np.array([SHELL_INNER[0] * rr * np.cos(ph), SHELL_INNER[1] * rr * np.sin(ph), z]))
    return np.array(sites)


def _conductivity(spec, centroids, dim):
    """Per-cell symmetric conductivity, packed (xx, xy, yy) in 2D and
    (xx, xy, xz, yy, yz, zz) in 3D."""
    nc = centroids.shape[0]
    if spec[0] == "iso":
        s = spec[1]
        if dim == 2:
            return np.tile(np.array([s, 0.0, s]), (nc, 1))
        return np.tile(np.array([s, 0.0, 0.0, s, 0.0, s]), (nc, 1))
    if spec[0] == "fibre_z":
        # D = sigma_t I + (sigma_l - sigma_t) f f^T, fibre angle rotating
        # linearly from -60 to +60 degrees along z (sigma_n = sigma_t).
        sl, st = spec[1], spec[2]
        th = np.deg2rad(-60.0 + 120.0 * centroids[:, 2])
        f = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)
        D = st * np.eye(3)[None] + (sl - st) * f[:, :, None] * f[:, None, :]
        return np.stack([D[:, 0, 0], D[:, 0, 1], D[:, 0, 2],
                         D[:, 1, 1], D[:, 1, 2], D[:, 2, 2]], axis=1)
    raise ValueError(spec)


def make_problem(name, n=None, steps=None, **overrides):
    """Build the input arrays of a named problem.

    ``n`` overrides the number of cells per axis (small variants for tests;
    for the shell, ``h`` overrides the voxel size); other keyword overrides
    replace config entries verbatim.
    """
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if cfg.get("kind") == "shell":
        return _make_shell(name, cfg, steps)
    if n is not None:
        if cfg["penalty"][0] == "fixed":
            # keep "10 p^2 / h" meaningful when the mesh is resized
            cfg["penalty"] = ("fixed", 10.0 * cfg["p"] ** 2 * n)
        cfg["n"] = n
        if "group" not in overrides:
            # keep only the grouping factors the smaller grid can take
            g, m = [], n
            for f in cfg["group"]:
                if m % f or m // f < 1:
                    break
                g.append(f)
                m //= f
            cfg["group"] = g
    if steps is not None:
        cfg["steps"] = steps
    dim, p = cfg["dim"], cfg["p"]
    xyz, cells = structured_mesh(dim, cfg["n"], cfg["jitter"], cfg["seed"])
    cen = cell_centroids(xyz, cells)
    nc = cells.shape[0]
    b = (p + 1) ** dim
    N = nc * b
    S = N_GATES[cfg["model"]]
    nodes = dof_nodes(xyz, cells, p).reshape(N, dim)
    U0 = np.zeros(N)
    W0 = np.zeros((S, N))
    if cfg["ic"] == "corner_disc":
        U0[np.linalg.norm(nodes, axis=1) < 0.1] = 1.0
    elif cfg["ic"] == "rest":
        if cfg["model"] == "bo":
            W0[0] = 1.0
            W0[1] = 1.0
    stim_mask = np.zeros(nc, dtype=bool)
    stim_amp, stim_tend = 0.0, 0.0
    if cfg["stim"] is not None and cfg["stim"][0] == "corner_block":
        _, edge, stim_amp, stim_tend = cfg["stim"]
        stim_mask = np.all(cen < edge, axis=1)
    elif cfg["stim"] is not None and cfg["stim"][0] == "box":
        _, lo, hi, stim_amp, stim_tend = cfg["stim"]
        stim_mask = np.all((cen > lo) & (cen < hi), axis=1)
    prob = dict(cfg)
    prob.update(name=name, xyz=xyz, cell_vtx=cells, n_cells=nc, b=b, N=N,
                S=S, D_cell=_conductivity(cfg["sigma"], cen, dim),
                U0=U0, W0=W0, stim_mask=stim_mask, stim_amp=stim_amp,
                stim_tend=stim_tend, model_id=MODEL_IDS[cfg["model"]],
                params=np.asarray(cfg["params"], dtype=np.float64),
                node_xyz=nodes)
    if cfg.get("sensors"):
        ns, seed = cfg["sensors"][:2]
        rng = np.random.default_rng(seed)
        if len(cfg["sensors"]) > 2:
            # distinct cells drawn from a band of centroid distances to the origin
            lo, hi = cfg["sensors"][2]
            r = np.linalg.norm(cen, axis=1)
            pool = np.flatnonzero((r >= lo) & (r <= hi))
            prob["sensor_cell"] = np.sort(rng.choice(pool, size=min(ns, len(pool)),
                                                     replace=False)).astype(np.int64)
        else:
            prob["sensor_cell"] = rng.integers(0, nc, size=ns).astype(np.int64)
        prob["sensor_ref"] = rng.uniform(0.0, 1.0, size=(len(prob["sensor_cell"]), dim))
        rng2 = np.random.default_rng(cfg["target_seed"])
        prob["s_true"] = np.exp(np.log(1.3) * rng2.standard_normal(nc))
    return prob


def probe_vector(n, seed):
    """Seeded unit vector of length n (entries uniform in [-1, 1] before
    normalisation), used to project a solution onto one number."""
    v = np.random.default_rng(seed).uniform(-1.0, 1.0, n)
    return v / np.linalg.norm(v)


def iapp_nodal(prob, t):
    """Applied current at DoF nodes at time t (piecewise constant per cell,
    switched on while t <= t_end)."""
    out = np.zeros(prob["N"])
    if prob["stim_amp"] and t <= prob["stim_tend"] + 1e-12:
        m = np.repeat(prob["stim_mask"], prob["b"])
        out[m] = prob["stim_amp"]
    return out


def _make_shell(name, cfg, steps):
    if steps is not None:
        cfg["steps"] = steps
    xyz, cells, surf = shell_mesh(cfg["h"], SHELL_OUTER, SHELL_INNER, 0.0, cfg["jitter"], cfg["seed"])
    cen = cell_centroids(xyz, cells)
    nc = cells.shape[0]
    p = cfg["p"]
    b = (p + 1) ** 3
    N = nc * b
    _, rad, amp, tend, sseed, nsites = cfg["stim"]
    sites = _stim_sites(nsites, sseed)
    masks = np.stack([np.linalg.norm(cen - s_, axis=1) < rad for s_ in sites])
    W0 = np.zeros((3, N))
    W0[0] = 1.0
    W0[1] = 1.0
    prob = dict(cfg)
    prob.update(name=name, xyz=xyz, cell_vtx=cells, n_cells=nc, b=b, N=N, S=3,
                D_cell=_shell_fibres(cen, cfg["sigma"][1], cfg["sigma"][2]),
                U0=np.zeros(N), W0=W0, stim_mask=masks[0], stim_masks=masks,
                stim_sites=sites, stim_amp=amp, stim_tend=tend,
                model_id=MODEL_IDS[cfg["model"]],
                params=np.asarray(cfg["params"], dtype=np.float64))
    return prob
