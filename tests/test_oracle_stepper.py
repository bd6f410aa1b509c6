"""Pins of the oracle's time stepper (section 3.1)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from workloads import make_problem
from oracle.ionic import gate_coeffs, ionic_current
from oracle.stepper import Simulation


def _uniform_run(model, prm, y0, ym1, T, n):
    pr = make_problem("c1", n=2, model=model, params=prm, dt=T / n)
    pr["params"] = np.asarray(prm, float)
    N = pr["N"]
    state = (np.full(N, y0[0]), np.full(N, ym1[0]),
             np.tile(np.asarray(y0[1:])[:, None], (1, N)),
             np.tile(np.asarray(ym1[1:])[:, None], (1, N)))
    sim = Simulation(pr)
    st, hist, stats = sim.run(n, 1e-14, state=state)
    return st


@pytest.mark.parametrize("model,prm,u0,w0,T", [
    ("fhn", [19.5, 0.13, 0.01, 0.5], 0.3, [0.0], 2.0),
    ("ap", [8.0, 0.15, 0.002], 0.3, [0.0], 2.0),
])
def test_uniform_data_is_second_order_ode_integrator(model, prm, u0, w0, T):
    """Spatially uniform data: the diffusion term vanishes, so each DoF
    integrates chi C du/dt = -chi I_ion(u, w), dw/dt = H(u, w).  Started
    from the exact history (U_{-1}, W_{-1}) = y(-dt), the scheme converges to
    scipy's reference integration at second order.  (The default start-up
    U_{-1} = U_0 is a reading that costs a first-order phase error.)"""
    prm = np.asarray(prm, float)

    def rhs(t, y):
        u = np.array([y[0]]); w = np.array(y[1:])[:, None]
        c1, c0 = gate_coeffs(model, prm, u)
        return np.concatenate([-ionic_current(model, prm, u, w),
                               (c1 * w + c0)[:, 0]])

    y0 = [u0] + list(w0)
    ref = solve_ivp(rhs, (0, T), y0, method="DOP853",
                    rtol=1e-12, atol=1e-14).y[:, -1]
    errs = []
    for n in (40, 80, 160):
        ym1 = solve_ivp(rhs, (0, -T / n), y0, method="DOP853",
                        rtol=1e-13, atol=1e-15).y[:, -1]
        st = _uniform_run(model, prm, y0, ym1, T, n)
        assert np.ptp(st[0]) < 1e-12
        errs.append(abs(st[0][0] - ref[0]))
    rate = np.log2(errs[1] / errs[2])
    assert 1.85 < rate < 2.3, (errs, rate)


def test_zero_conductivity_decouples_dofs():
    """sigma = 0 gives A = 0, so (3/(2dt)) chi C M U' = M f reduces to the
    nodal recurrence U' = 2 dt f / (3 chi C) at every DoF."""
    pr = make_problem("c1", n=4, sigma=("iso", 0.0))
    rng = np.random.default_rng(7)
    pr["U0"] = rng.uniform(0, 1, pr["N"])
    sim = Simulation(pr)
    st, hist, _ = sim.run(4, 1e-14)
    U, Um = pr["U0"].copy(), pr["U0"].copy()
    W, Wm = pr["W0"].copy(), pr["W0"].copy()
    k, a, eps, gam = pr["params"]
    dt = pr["dt"]
    for n in range(4):
        us = 2 * U - Um
        Wn = (4 * W - Wm + 2 * dt * eps * us) / (3 + 2 * dt * eps * gam)
        g = k * us * (us - a) * (us - 1) + Wn[0]
        f = (4 * U - Um) / (2 * dt) - g
        U, Um = 2 * dt * f / 3, U
        W, Wm = Wn, W
        assert np.allclose(hist[n], U, rtol=1e-12, atol=1e-13)


def test_zero_conductivity_with_applied_current_and_scalings():
    """sigma = 0 with chi, C_m != 1 and a constant applied current on part of
    the mesh: c_M M U' = M f with c_M = 3 chi C_m / (2 dt) gives, per DoF,
    U' = 2 dt f / (3 chi C_m) with
    f = chi C_m / (2 dt) (4 U - U_prev) + I_app - chi g (eq. fully_discrete,
    ionic current interpolation)."""
    chi, Cm, amp = 2.5, 0.8, 0.7
    pr = make_problem("c1", n=4, sigma=("iso", 0.0), chi=chi, Cm=Cm)
    rng = np.random.default_rng(9)
    pr["U0"] = rng.uniform(0, 1, pr["N"])
    stim = np.zeros(pr["n_cells"], dtype=bool)
    stim[[0, 3, 5, 10]] = True
    iapp = np.repeat(stim, pr["b"]) * amp
    sim = Simulation(pr)
    st, hist, _ = sim.run(4, 1e-14, iapp_fn=lambda t: iapp)
    U, Um = pr["U0"].copy(), pr["U0"].copy()
    W, Wm = pr["W0"].copy(), pr["W0"].copy()
    k, a, eps, gam = pr["params"]
    dt = pr["dt"]
    for n in range(4):
        us = 2 * U - Um
        Wn = (4 * W - Wm + 2 * dt * eps * us) / (3 + 2 * dt * eps * gam)
        g = k * us * (us - a) * (us - 1) + Wn[0]
        f = chi * Cm / (2 * dt) * (4 * U - Um) + iapp - chi * g
        U, Um = 2 * dt * f / (3 * chi * Cm), U
        W, Wm = Wn, W
        assert np.allclose(hist[n], U, rtol=1e-12, atol=1e-13)
