"""Discrete adjoint of the semi-implicit time stepper with respect to per-cell
conductivity scalings s_K (D_K -> s_K D_K), for the sensor misfit
    L(s) = sum_{n=1..N} sum_k (e_k^T U_n - V_{k,n})^2,
where e_k^T U evaluates the DG field of cell K_k at reference point xi_k.

A(s) is linear in s: every term of a_h (section 3) carries exactly one
conductivity tensor, the penalty uses the mean of the two sides' n^T D n, so
A(s) = sum_K s_K G_K with G_K the cell stiffness of K plus, on every face of
K, the part of the face matrix that K's tensor multiplies.  Only the linear
solve depends on s.

Reverse step n (forward: state_n -> (U_{n+1}, W_{n+1})), given the adjoints
Ubar_{n+1}, Wbar_{n+1} accumulated from the loss and from later steps:
  lambda = A_0^-1 Ubar_{n+1}                 (A_0 symmetric)
  dL/ds_K -= lambda^T G_K U_{n+1}
  fbar = M lambda;  Ubar_n += 4 cU fbar;  Ubar_{n-1} -= cU fbar;  gbar = -chi fbar
  Wtot = Wbar_{n+1} + dI/dw gbar
  Ustar_bar = dI/du gbar + Wtot * 2 dt (c0' + W_{n+1} c1') / (3 - 2 dt c1)
  Wbar_n += 4 Wtot / (3 - 2 dt c1);  Wbar_{n-1} -= Wtot / (3 - 2 dt c1)
  Ubar_n += 2 Ustar_bar;  Ubar_{n-1} -= Ustar_bar
The first step's history U_{-1} = U_0 is fixed data.  Forward states are
recomputed segment by segment from checkpoints.

Pins (tests/test_oracle_adjoint.py): central finite differences of the
oracle's forward loss along random directions; the evaluation functionals
e_k reproduce Q_p polynomials of the sensor cell's reference coordinates and
linear physical fields at the mapped sensor points.
"""
import numpy as np
import scipy.sparse as sp

from .assemble import (cell_matrices, face_matrices, interior_faces, unpack_sym,
                       system_matrix)
from .basis import tensor_basis
from .ionic import gate_coeffs, ionic_current
from .mg import pcg
from .stepper import Simulation


def ionic_derivatives(model, prm, u, w):
    """(dI/du [N], dI/dw [S,N], dc1/du [S,N], dc0/du [S,N]) at (u, w)."""
    if model == "fhn":
        k, a, eps, gam = prm
        dIu = k * (3 * u * u - 2 * (a + 1) * u + a)
        return dIu, np.ones_like(w), np.zeros_like(w), np.full_like(w, eps)
    if model == "ap":
        k, a, eps0 = prm
        dIu = k * (3 * u * u - 2 * (a + 1) * u + a) + w[0]
        dIw = u[None].copy()
        dc0 = (-eps0 * k * (2 * u - a - 1))[None]
        return dIu, dIw, np.zeros_like(w), dc0
    raise NotImplementedError("adjoint implemented for FHN and Aliev-Panfilov")


def sensor_matrix(prob):
    """Sparse E with (E U)_k = e_k^T U."""
    p, d, b, N = prob["p"], prob["dim"], prob["b"], prob["N"]
    phi, _ = tensor_basis(p, d, prob["sensor_ref"])
    rows = np.repeat(np.arange(len(prob["sensor_cell"])), b)
    cols = (prob["sensor_cell"][:, None] * b + np.arange(b)[None]).ravel()
    return sp.csr_matrix((phi.ravel(), (rows, cols)), shape=(len(prob["sensor_cell"]), N))


def derivative_blocks(prob):
    """Cell stiffness S_K (unscaled D) and the per-side face matrices X+/X-
    (2b x 2b over [K+ DoFs, K- DoFs]) with faces (plus, minus)."""
    xyz, cells, p = prob["xyz"], prob["cell_vtx"], prob["p"]
    d = xyz.shape[1]
    D = unpack_sym(prob["D_cell"], d)
    X = xyz[cells]
    _, S, vol = cell_matrices(X, D, p)
    plus, minus, axis = interior_faces(cells, d)
    Xp = np.zeros((len(plus), 2 * prob["b"], 2 * prob["b"]))
    Xm = np.zeros_like(Xp)
    zero = np.zeros_like(D)
    for k in range(d):
        sel = np.flatnonzero(axis == k)
        fp, fm = plus[sel], minus[sel]
        Xp[sel] = face_matrices(X[fp], X[fm], D[fp], zero[fm], k, vol[fp], vol[fm], p,
                                prob["penalty"])
        Xm[sel] = face_matrices(X[fp], X[fm], zero[fp], D[fm], k, vol[fp], vol[fm], p,
                                prob["penalty"])
    return S, plus, minus, Xp, Xm


def grad_contribution(prob, blocks, lam, U):
    """-lambda^T G_K U for every cell K."""
    S, plus, minus, Xp, Xm = blocks
    b, nc = prob["b"], prob["n_cells"]
    L = lam.reshape(nc, b)
    V = U.reshape(nc, b)
    g = -np.einsum("ni,nij,nj->n", L, S, V)
    lf = np.concatenate([L[plus], L[minus]], axis=1)
    uf = np.concatenate([V[plus], V[minus]], axis=1)
    np.add.at(g, plus, -np.einsum("fi,fij,fj->f", lf, Xp, uf))
    np.add.at(g, minus, -np.einsum("fi,fij,fj->f", lf, Xm, uf))
    return g


class AdjointProblem:
    """Forward loss and its adjoint gradient at scalings s (FP64 oracle)."""

    def __init__(self, prob, targets, steps, tol=1e-13, checkpoint=10):
        self.prob, self.targets, self.steps = prob, targets, steps
        self.tol, self.ck = tol, checkpoint
        self.E = sensor_matrix(prob)
        self.blocks = derivative_blocks(prob)

    def forward(self, s, keep=False):
        pr = self.prob
        sim = Simulation(pr, scale=s)
        state = (pr["U0"].copy(), pr["U0"].copy(), pr["W0"].copy(), pr["W0"].copy())
        loss, ckpts = 0.0, {}
        for n in range(self.steps):
            if n % self.ck == 0:
                ckpts[n] = tuple(a.copy() for a in state)
            state, _ = sim.step(state, (n + 1) * pr["dt"], self.tol)
            r = self.E @ state[0] - self.targets[n]
            loss += float(r @ r)
        return (loss, sim, ckpts) if keep else loss

    def gradient(self, s):
        pr = self.prob
        loss, sim, ckpts = self.forward(s, keep=True)
        dt, chi, cU = pr["dt"], pr["chi"], pr["chi"] * pr["Cm"] / (2 * pr["dt"])
        N, S = pr["N"], pr["S"]
        grad = np.zeros(pr["n_cells"])
        Ub = {}   # adjoint accumulators keyed by time index
        Wb = {}
        for seg in sorted(ckpts, reverse=True):
            # replay the segment, keeping every state
            states = [ckpts[seg]]
            for n in range(seg, min(seg + self.ck, self.steps)):
                st, _ = sim.step(states[-1], (n + 1) * dt, self.tol)
                states.append(st)
            for n in reversed(range(seg, min(seg + self.ck, self.steps))):
                Un, Unm1, Wn, Wnm1 = states[n - seg]
                Unew, _, Wnew, _ = states[n - seg + 1]
                ub = Ub.pop(n + 1, np.zeros(N))
                ub = ub + 2.0 * (self.E.T @ (self.E @ Unew - self.targets[n]))
                wb = Wb.pop(n + 1, np.zeros((S, N)))
                lam, _ = pcg(sim.A0, ub, np.zeros(N), sim.mg, self.tol)
                grad += grad_contribution(pr, self.blocks, lam, Unew)
                fb = sim.M @ lam
                gb = -chi * fb
                us = 2.0 * Un - Unm1
                c1, c0 = gate_coeffs(pr["model"], pr["params"], us)
                dIu, dIw, dc1, dc0 = ionic_derivatives(pr["model"], pr["params"], us, Wnew)
                den = 3.0 - 2.0 * dt * c1
                wtot = wb + dIw * gb
                usb = dIu * gb + (wtot * 2.0 * dt * (dc0 + Wnew * dc1) / den).sum(axis=0)
                Ub[n] = Ub.get(n, np.zeros(N)) + 4.0 * cU * fb + 2.0 * usb
                Ub[n - 1] = Ub.get(n - 1, np.zeros(N)) - cU * fb - usb
                Wb[n] = Wb.get(n, np.zeros((S, N))) + 4.0 * wtot / den
                Wb[n - 1] = Wb.get(n - 1, np.zeros((S, N))) - wtot / den
        return loss, grad


def make_targets(prob, steps, s_true, tol=1e-13):
    """Sensor values of the forward run at the true scalings, [steps, n_sensors]."""
    E = sensor_matrix(prob)
    sim = Simulation(prob, scale=s_true)
    st = (prob["U0"].copy(), prob["U0"].copy(), prob["W0"].copy(), prob["W0"].copy())
    out = []
    for n in range(steps):
        st, _ = sim.step(st, (n + 1) * prob["dt"], tol)
        out.append(E @ st[0])
    return np.array(out)
