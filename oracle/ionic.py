"""Ionic models evaluated at DoFs and their BDF2 gate update (section 2.2:
FitzHugh-Nagumo and Bueno-Orovio; section 3.1: ionic ODEs solved by BDF2 at
every DoF, current evaluated at the DoFs (ICI)).

Every model used here has gate dynamics that are affine in each gate for a
fixed potential, dw/dt = c1(u) w + c0(u), so the BDF2 step
(3 W' - 4 W_n + W_{n-1}) / (2 dt) = c1(U*) W' + c0(U*) has a closed form.
The potential driving the gates is the extrapolation U* = 2 U_n - U_{n-1}.

Readings:
* FHN: I_ion = k u (u - a)(u - 1) + w, dw/dt = eps (u - Gamma w); parameter
  vector [k, a, eps, Gamma];
* Aliev-Panfilov (not in the paper): I_ion = k u (u-a)(u-1) + u v,
  dv/dt = eps0 (-v - k u (u - a - 1)) (mu1 = 0); vector [k, a, eps0];
* Bueno-Orovio: the printed Heaviside variants are read as: H^-_{V1} ->
  sharp H at V_1m; H^-_{V2} -> smooth H (k_2) at V_2m; w0_inf uses sharp H at
  V_1m; w2_inf = smooth H (k_3) at V_3; the second so-term uses smooth H
  (k_so) at V_so; the first so-term uses (u - u_o) with u_o = 0; a sharp H at
  its threshold equals 1/2.  "parity unpinned" for the parameter set itself.

Pins (tests/test_oracle_ionic.py): hand-computed values at chosen (u, w),
rest states, closed-form gate relaxation, second-order convergence of the
time stepper on spatially uniform data.
"""
import numpy as np

from workloads.configs import BO_PARAM_NAMES


def H_sharp(z):
    return np.where(z > 0, 1.0, np.where(z < 0, 0.0, 0.5))


def H_smooth(z, k):
    return 0.5 * (1.0 + np.tanh(k * z))


def gate_coeffs(model, prm, u):
    """(c1, c0) of shape [S, N] with dw/dt = c1 * w + c0."""
    if model == "fhn":
        k, a, eps, gam = prm
        return (np.full((1,) + u.shape, -eps * gam), (eps * u)[None])
    if model == "ap":
        k, a, eps0 = prm
        return (np.full((1,) + u.shape, -eps0),
                (-eps0 * k * u * (u - a - 1.0))[None])
    if model == "bo":
        P = dict(zip(BO_PARAM_NAMES, prm))
        H1 = H_sharp(u - P["V_1"])
        H2 = H_sharp(u - P["V_2"])
        H1m = H_sharp(u - P["V_1m"])
        H2m = H_smooth(u - P["V_2m"], P["k_2"])
        Ho = H_sharp(u - P["V_o"])
        a0 = (1.0 - H1) / (H1m * (P["tau_1m2"] - P["tau_1m1"]) + P["tau_1m1"])
        a1 = (1.0 - H2) / (H2m * (P["tau_2m2"] - P["tau_2m1"]) + P["tau_2m1"])
        a2 = 1.0 / (H2 * (P["tau_3m2"] - P["tau_3m1"]) + P["tau_3m1"])
        b0 = -H1 / P["tau_1p"]
        b1 = -H2 / P["tau_2p"]
        b2 = np.zeros_like(u)
        w0i = 1.0 - H1m
        w1i = Ho * (P["w_inf_star"] - 1.0 + u / P["tau_2inf"]) + 1.0 - u / P["tau_2inf"]
        w2i = H_smooth(u - P["V_3"], P["k_3"])
        c1 = np.stack([b0 - a0, b1 - a1, b2 - a2])
        c0 = np.stack([a0 * w0i, a1 * w1i, a2 * w2i])
        return c1, c0
    raise ValueError(model)


def ionic_current(model, prm, u, w):
    """I_ion(u, w) at DoFs; w has shape [S, N]."""
    if model == "fhn":
        k, a, eps, gam = prm
        return k * u * (u - a) * (u - 1.0) + w[0]
    if model == "ap":
        k, a, eps0 = prm
        return k * u * (u - a) * (u - 1.0) + u * w[0]
    if model == "bo":
        P = dict(zip(BO_PARAM_NAMES, prm))
        H1 = H_sharp(u - P["V_1"])
        H2 = H_sharp(u - P["V_2"])
        Ho = H_sharp(u - P["V_o"])
        Hso = H_smooth(u - P["V_so"], P["k_so"])
        I_fi = -H1 * (u - P["V_1"]) * (P["V_hat"] - u) * w[0] / P["tau_fi"]
        I_si = -H2 * w[1] * w[2] / P["tau_si"]
        I_so = ((1.0 - H2) * (u - P["u_o"]) / (Ho * (P["tau_o2"] - P["tau_o1"]) + P["tau_o1"])
                + H2 / (Hso * (P["tau_so2"] - P["tau_so1"]) + P["tau_so1"]))
        return I_fi + I_si + I_so
    raise ValueError(model)


def gate_step(model, prm, ustar, Wn, Wnm1, dt, bdf=2):
    """W_{n+1} from the affine gate ODE discretised by BDF2 (or backward
    Euler when bdf == 1), driven by ustar."""
    c1, c0 = gate_coeffs(model, prm, ustar)
    if bdf == 2:
        return (4.0 * Wn - Wnm1 + 2.0 * dt * c0) / (3.0 - 2.0 * dt * c1)
    return (Wn + dt * c0) / (1.0 - dt * c1)
