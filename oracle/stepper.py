"""Semi-implicit time stepping of the monodomain system (section 3.1,
eq. fully_discrete and the three-step procedure after it).

Per step, given (U_n, U_{n-1}, W_n, W_{n-1}):
  1. U* = 2 U_n - U_{n-1}; W_{n+1} from the BDF2 gate update at U*;
  2. nodal ionic current g = I_ion(U*, W_{n+1}); with ICI the load vector is
     M f for the nodal field
     f = chi C_m / (2 dt) (4 U_n - U_{n-1}) + I_app(t_{n+1}) - chi g;
  3. solve (3 chi C_m / (2 dt) M + A) U_{n+1} = M f by PCG with one V-cycle
     per iteration, warm-started from U_n.
Reading: the first step uses U_{-1} = U_0 and W_{-1} = W_0, so the single
assembled matrix serves every step.  bdf=1 selects backward Euler
(matrix chi C_m / dt M + A, U* = U_n).

Pins (tests/test_oracle_stepper.py): spatially uniform data reduces to the
per-DoF ODE integrator (second-order convergence against a fine reference
integration); zero conductivity makes every DoF independent, including the
applied-current term and the chi, C_m scalings of the load vector.
"""
import time

import numpy as np

from .assemble import system_matrix
from .hierarchy import build_hierarchy
from .ionic import gate_step, ionic_current
from .mg import VCycle, pcg


class Simulation:
    """Holds the assembled operators and the preconditioner of a problem."""

    def __init__(self, prob, bdf=2, lam_override=None, scale=None,
                 flexible=False):
        self.prob = prob
        self.bdf = bdf
        self.A0, self.M, self.A, self.cM = system_matrix(prob, scale, bdf)
        self.hier = build_hierarchy(prob)
        self.mg = VCycle(self.A0, self.hier["P"], lam_override=lam_override)
        self.flexible = flexible

    def rhs(self, Un, Unm1, g, t_next, iapp=None):
        pr = self.prob
        c = pr["chi"] * pr["Cm"]
        if self.bdf == 2:
            f = c / (2.0 * pr["dt"]) * (4.0 * Un - Unm1) - pr["chi"] * g
        else:
            f = c / pr["dt"] * Un - pr["chi"] * g
        if iapp is not None:
            f = f + iapp
        return self.M @ f

    def step(self, state, t_next, tol, iapp=None, max_it=500, tol_mode="rel"):
        pr = self.prob
        Un, Unm1, Wn, Wnm1 = state
        ustar = 2.0 * Un - Unm1 if self.bdf == 2 else Un
        Wnew = gate_step(pr["model"], pr["params"], ustar, Wn, Wnm1, pr["dt"],
                         self.bdf)
        g = ionic_current(pr["model"], pr["params"], ustar, Wnew)
        b = self.rhs(Un, Unm1, g, t_next, iapp)
        Unew, st = pcg(self.A0, b, Un, self.mg, tol, max_it, self.flexible, tol_mode)
        return (Unew, Un, Wnew, Wn), st

    def run(self, steps, tol, iapp_fn=None, state=None, record=True, tol_mode="rel"):
        pr = self.prob
        if state is None:
            state = (pr["U0"].copy(), pr["U0"].copy(), pr["W0"].copy(),
                     pr["W0"].copy())
        hist, stats = [], []
        for n in range(steps):
            t = (n + 1) * pr["dt"]
            iapp = iapp_fn(t) if iapp_fn is not None else None
            t0 = time.perf_counter()
            state, st = self.step(state, t, tol, iapp, tol_mode=tol_mode)
            st["wall"] = time.perf_counter() - t0
            stats.append(st)
            if record:
                hist.append(state[0].copy())
        return state, hist, stats
