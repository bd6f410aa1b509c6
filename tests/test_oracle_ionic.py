"""Pins of the oracle's ionic models and BDF2 gate update (section 2.2 and
section 3.1)."""
import numpy as np
import pytest

from workloads.configs import BO_EPI, BO_PARAM_NAMES
from oracle.ionic import gate_coeffs, gate_step, ionic_current

FHN = np.array([19.5, 0.13, 0.01, 0.5])
AP = np.array([8.0, 0.15, 0.002])
BO = np.array([BO_EPI[k] for k in BO_PARAM_NAMES])


def test_fhn_hand_values_and_cubic_roots():
    u = np.array([0.5]); w = np.array([[0.2]])
    # 19.5 * 0.5 * 0.37 * (-0.5) + 0.2
    assert abs(ionic_current("fhn", FHN, u, w)[0] - (-1.60375)) < 1e-14
    roots = np.array([0.0, 0.13, 1.0])
    assert np.allclose(ionic_current("fhn", FHN, roots, np.zeros((1, 3))), 0, atol=1e-15)
    c1, c0 = gate_coeffs("fhn", FHN, u)
    # dw/dt = eps (u - Gamma w) at w = 0.2: 0.01 * (0.5 - 0.1)
    assert abs((c1 * 0.2 + c0)[0, 0] - 0.004) < 1e-16


def test_aliev_panfilov_hand_values():
    u = np.array([0.5]); v = np.array([[0.1]])
    # 8 * 0.5 * 0.35 * (-0.5) + 0.5 * 0.1
    assert abs(ionic_current("ap", AP, u, v)[0] - (-0.65)) < 1e-14
    c1, c0 = gate_coeffs("ap", AP, u)
    # dv/dt = 0.002 * (-0.1 - 8 * 0.5 * (0.5 - 1.15)) = 0.002 * 2.5
    assert abs((c1 * 0.1 + c0)[0, 0] - 0.005) < 1e-16


def test_bueno_orovio_rest_state_and_hand_values():
    u = np.array([0.0])
    w = np.array([[1.0], [1.0], [0.0]])
    assert ionic_current("bo", BO, u, w)[0] == 0.0
    c1, c0 = gate_coeffs("bo", BO, u)
    rate = c1[:, 0] * w[:, 0] + c0[:, 0]
    assert rate[0] == 0.0 and rate[1] == 0.0
    # w2 relaxes to the smooth Heaviside (k_3 = 2.0994 at V_3 = 0.9087) of 0
    assert abs(-c0[2, 0] / c1[2, 0] - 0.021553043080280776) < 1e-15
    # excited point u = 1, w = (0.5, 0.8, 0.3)
    u = np.array([1.0]); w = np.array([[0.5], [0.8], [0.3]])
    I_fi = -0.7 * 0.58 * 0.5 / 0.11
    I_si = -0.08355673153918462
    I_so = 0.11538644066905983
    assert abs(ionic_current("bo", BO, u, w)[0] - (I_fi + I_si + I_so)) < 1e-13
    # the sharp Heaviside at its threshold is one half
    c1a, _ = gate_coeffs("bo", BO, np.array([BO_EPI["V_1"]]))
    assert abs(c1a[0, 0] - (-0.5 / 1.4506 - 0.5 / 1150.0)) < 1e-15


@pytest.mark.parametrize("model,prm,u", [("fhn", FHN, 0.4), ("ap", AP, 0.6),
                                         ("bo", BO, 0.2), ("bo", BO, 0.95)])
def test_bdf2_gate_update_second_order(model, prm, u):
    """At fixed u the gate ODE is linear with exact solution
    w_inf + (w0 - w_inf) exp(c1 t); the BDF2 recursion started from the exact
    history W_{-1} = w(-dt) converges to it at second order."""
    uu = np.array([u])
    c1, c0 = gate_coeffs(model, prm, uu)
    S = c1.shape[0]
    w0 = np.full((S, 1), 0.3)
    T = 20.0 / max(1e-3, np.abs(c1).max())
    winf = -c0 / c1
    exact = winf + (w0 - winf) * np.exp(c1 * T)
    errs = []
    for n in (50, 100, 200):
        dt = T / n
        Wn, Wm = w0.copy(), winf + (w0 - winf) * np.exp(-c1 * dt)
        for _ in range(n):
            Wn, Wm = gate_step(model, prm, uu, Wn, Wm, dt), Wn
        errs.append(np.abs(Wn - exact).max())
    rate = np.log2(errs[1] / errs[2])
    assert rate > 1.8 or errs[2] < 1e-13, (errs, rate)
