"""Agglomerated multigrid preconditioner and PCG (section 5.1: inherited
operators A_{l+1} = P^T A_l P, Algorithm 3; section 6: Chebyshev-accelerated
Jacobi smoother of degree 3 with Lanczos eigenvalue estimates, 3 pre- and
post-smoothing steps, one V-cycle per PCG iteration).

Readings (listed in the design notes):
* Lanczos: m = 20 steps on D^-1/2 A D^-1/2 without reorthogonalisation,
  start vector v_i = frac((i+1) * 0.6180339887498949) - 0.5, stop early when
  beta < 1e-14 (the scaled operator has unit diagonal) or after n steps;
  lambda_hi = 1.2 * theta_max,
  lambda_lo = lambda_hi / 20  ("parity unpinned": constants by convention);
* Chebyshev: Saad, Iterative Methods for Sparse Linear Systems, the
  Chebyshev acceleration algorithm preconditioned by D^-1; "degree 3 with 3
  smoothing steps" = the degree-3 recurrence restarted 3 times, each restart
  from the true residual b - A x;
* Jacobi matrix D: the diagonal of A_l (section 6, the paper's choice) or,
  as an option, the cells' b x b diagonal blocks ("point-block" Jacobi);
  the block variant's Lanczos runs on L^-1 A L^-T with D_K = L_K L_K^T per
  cell, which is similar to D^-1 A and also has a unit diagonal;
* coarsest level: exact dense Cholesky solve;
* PCG stops when ||r_k||_2 <= tol * ||r_0||_2 with r_0 from the warm start;
  the iteration count is the number of A applies inside the loop.

Pins (tests/test_oracle_mg.py): Galerkin symmetry and kernel, Lanczos bound
and accuracy against dense eigenvalues (generalised eigenvalues of (A, D)
for the block variant), Chebyshev error propagator equals the closed-form
Chebyshev polynomial (both Jacobi variants), V-cycle symmetry and positivity,
special cases (no smoothing -> P A_c^-1 P^T; one level -> exact inverse), PCG
against dense solves.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def galerkin(A, P):
    """A_{l+1} = P^T A_l P."""
    return (P.T @ A @ P).tocsr()


def lanczos_start(n):
    i = np.arange(n, dtype=np.float64)
    t = (i + 1.0) * 0.6180339887498949
    return t - np.floor(t) - 0.5


def lanczos_theta_max(A, diag, m=20):
    """Largest Ritz value of m Lanczos steps on D^-1/2 A D^-1/2."""
    n = A.shape[0]
    s = 1.0 / np.sqrt(diag)
    v = lanczos_start(n)
    v /= np.linalg.norm(v)
    v_prev = np.zeros(n)
    alphas, betas = [], []
    beta = 0.0
    for j in range(min(m, n)):
        w = s * (A @ (s * v)) - beta * v_prev
        a = w @ v
        w = w - a * v
        alphas.append(a)
        beta = np.linalg.norm(w)
        if beta < 1e-14 or j == min(m, n) - 1:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) \
        + np.diag(betas[:len(alphas) - 1], -1)
    return float(np.linalg.eigvalsh(T).max())


def diagonal_blocks(A, b):
    """The cells' b x b diagonal blocks of A (n_cells x b x b)."""
    C = A.tocoo()
    keep = (C.row // b) == (C.col // b)
    r, c = C.row[keep], C.col[keep]
    Dk = np.zeros((A.shape[0] // b, b, b))
    np.add.at(Dk, (r // b, r % b, c % b), C.data[keep])
    return Dk


def cell_block_inverse(A, b):
    """D^-1 for the cell-block Jacobi variant: the inverse of every diagonal
    block, as a block-diagonal sparse matrix."""
    return sp.block_diag(list(np.linalg.inv(diagonal_blocks(A, b))), format="csr")


def lanczos_theta_max_block(A, b, m=20):
    """Largest Ritz value of m Lanczos steps on L^-1 A L^-T, where
    D_K = L_K L_K^T are the Cholesky factors of the cells' diagonal blocks;
    the same start vector and stopping rule as the point variant."""
    n = A.shape[0]
    Linv = np.linalg.inv(np.linalg.cholesky(diagonal_blocks(A, b)))
    nb = n // b

    def op(v):
        y = np.einsum("kji,kj->ki", Linv, v.reshape(nb, b)).ravel()       # L^-T v
        return np.einsum("kij,kj->ki", Linv, (A @ y).reshape(nb, b)).ravel()  # L^-1 (A y)

    v = lanczos_start(n)
    v /= np.linalg.norm(v)
    v_prev = np.zeros(n)
    alphas, betas = [], []
    beta = 0.0
    for j in range(min(m, n)):
        w = op(v) - beta * v_prev
        a = w @ v
        w = w - a * v
        alphas.append(a)
        beta = np.linalg.norm(w)
        if beta < 1e-14 or j == min(m, n) - 1:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) \
        + np.diag(betas[:len(alphas) - 1], -1)
    return float(np.linalg.eigvalsh(T).max())


def chebyshev(A, dinv, b, x, lam_lo, lam_hi, degree=3, sweeps=3):
    """Chebyshev-accelerated Jacobi: ``sweeps`` restarts of the degree-k
    recurrence on the interval [lam_lo, lam_hi] of D^-1 A.  ``dinv`` is the
    inverse diagonal (a vector) or the block-diagonal D^-1 (a sparse
    matrix)."""
    jac = (lambda r: dinv @ r) if sp.issparse(dinv) else (lambda r: dinv * r)
    theta = 0.5 * (lam_hi + lam_lo)
    delta = 0.5 * (lam_hi - lam_lo)
    sigma1 = theta / delta
    x = x.copy()
    for _ in range(sweeps):
        r = b - A @ x
        d = jac(r) / theta
        rho = 1.0 / sigma1
        for i in range(degree):
            x = x + d
            if i == degree - 1:
                break
            r = r - A @ d
            rho_new = 1.0 / (2.0 * sigma1 - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * jac(r)
            rho = rho_new
    return x


class VCycle:
    """One V-cycle of agglomerated multigrid as a linear operator."""

    def __init__(self, A0, P, degree=3, sweeps=3, lanczos_m=20,
                 lam_override=None, safety=1.2, smooth_range=20.0,
                 jacobi="point", b=None):
        """jacobi: "point" (inverse diagonal) or "cell_block" (inverse b x b
        diagonal blocks; b is the block size of every level)."""
        if jacobi not in ("point", "cell_block"):
            raise ValueError(jacobi)
        self.A = [A0.tocsr()]
        self.P = P
        for Pl in P:
            self.A.append(galerkin(self.A[-1], Pl))
        self.L = len(self.A)
        if jacobi == "point":
            self.dinv = [1.0 / Al.diagonal() for Al in self.A]
        else:
            self.dinv = [cell_block_inverse(Al, b) for Al in self.A[:-1]] + [None]
        self.lam = []
        for l in range(self.L - 1):
            if lam_override is not None:
                lo, hi = lam_override[l]
            else:
                th = (lanczos_theta_max(self.A[l], self.A[l].diagonal(), lanczos_m) if jacobi == "point"
                      else lanczos_theta_max_block(self.A[l], b, lanczos_m))
                hi = safety * th
                lo = hi / smooth_range
            self.lam.append((lo, hi))
        self.degree, self.sweeps = degree, sweeps
        Ac = self.A[-1].toarray()
        self.chol = sla.cho_factor(Ac, lower=True)

    def coarse_solve(self, b):
        return sla.cho_solve(self.chol, b)

    def apply(self, b, level=0):
        if level == self.L - 1:
            return self.coarse_solve(b)
        A, dinv = self.A[level], self.dinv[level]
        lo, hi = self.lam[level]
        x = np.zeros_like(b)
        x = chebyshev(A, dinv, b, x, lo, hi, self.degree, self.sweeps)
        r = b - A @ x
        e = self.apply(self.P[level].T @ r, level + 1)
        x = x + self.P[level] @ e
        x = chebyshev(A, dinv, b, x, lo, hi, self.degree, self.sweeps)
        return x

    __call__ = apply


def pcg(A, b, x0, prec, tol, max_it=500, flexible=False, tol_mode="rel"):
    """Preconditioned conjugate gradients from the warm start x0.

    Stops when ||r_k|| <= tol ||r_0|| (tol_mode "rel"), or ||r_k|| <= tol
    ("abs", the absolute residual of the paper's two-dimensional test in
    section 6).  Returns (x, stats) with stats = dict(its, r0, rfin,
    converged).
    """
    x = x0.copy()
    r = b - A @ x
    r0 = np.linalg.norm(r)
    thresh = tol if tol_mode == "abs" else tol * r0
    if r0 == 0.0 or (tol_mode == "abs" and r0 <= thresh):
        return x, dict(its=0, r0=r0, rfin=r0, converged=True)
    z = prec(r)
    p = z.copy()
    gamma = r @ z
    its = 0
    rn = r0
    while its < max_it:
        q = A @ p
        pq = p @ q
        if pq <= 0 or gamma <= 0:
            raise FloatingPointError("PCG breakdown: operator not SPD")
        alpha = gamma / pq
        x = x + alpha * p
        r = r - alpha * q
        its += 1
        rn = np.linalg.norm(r)
        if rn <= thresh:
            return x, dict(its=its, r0=r0, rfin=rn, converged=True)
        z_old = z
        z = prec(r)
        gamma_new = r @ z
        if flexible:
            beta = (gamma_new - r @ z_old) / gamma
        else:
            beta = gamma_new / gamma
        p = z + beta * p
        gamma = gamma_new
    return x, dict(its=its, r0=r0, rfin=rn, converged=False)
