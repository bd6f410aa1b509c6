"""Gradient of a sensor misfit with respect to per-cell conductivity scalings,
as a torch.autograd.Function over the GPU time stepper.

Forward: set up the solver for D_K -> s_K D_K, run the semi-implicit steps,
accumulate L = sum_n sum_k (e_k^T U_n - V_{k,n})^2, keep the state every
`checkpoint` steps.  Backward (discrete adjoint, reverse order): replay each
segment from its checkpoint, then for every step
  Ubar_{n+1} += dL_{n+1}/dU;  lambda = A_0^-1 Ubar_{n+1} (same PCG and V-cycle,
  A_0 is symmetric);  grad_K -= lambda^T dA/ds_K U_{n+1};
  reverse of the ionic update and load vector into Ubar_n, Ubar_{n-1},
  Wbar_n, Wbar_{n-1}.
Every operation is a library call; this module only allocates tensors and
orders the calls.
"""
import numpy as np
import torch

from . import api, problem


def _zeros(n):
    return torch.zeros(n, dtype=torch.float64, device="cuda")


def _fresh_state(prob):
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")
    return api.State(dev(prob["U0"]), dev(prob["U0"]), dev(prob["W0"].ravel()),
                     dev(prob["W0"].ravel()), _zeros(prob["N"]))


def _copy_state(st):
    return api.State(st.U.clone(), st.Uprev.clone(), st.W.clone(), st.Wprev.clone(),
                     st.g.clone())


class SensorMisfit(torch.autograd.Function):
    """loss = SensorMisfit.apply(s, prob, targets, steps, tol, checkpoint, precision)."""

    @staticmethod
    def forward(ctx, s, prob, targets, steps, tol, checkpoint, precision):
        s_host = s.detach().double().cpu().numpy()
        # hierarchy on the GPU (the fine blocks and dA/ds_K come from the host
        # assembly when the adjoint is requested), memory from torch
        h, solver = problem.build(prob, precision=precision, cell_scale=s_host, adjoint=True,
                                  setup="device", allocator="torch")
        api.set_sensors(solver, prob["sensor_cell"], prob["sensor_ref"])
        st = _fresh_state(prob)
        loss = _zeros(1)
        ckpts = {}
        its = []
        for n in range(steps):
            if n % checkpoint == 0:
                ckpts[n] = _copy_state(st)
            r = api.time_step(solver, st, (n + 1) * prob["dt"], tol=tol)
            its.append(r["its"])
            api.sensor_misfit(solver, st.U, targets[n], None, loss)
        ctx.solver, ctx.hier, ctx.ckpts = solver, h, ckpts
        ctx.prob, ctx.targets, ctx.steps, ctx.tol, ctx.ck = prob, targets, steps, tol, checkpoint
        ctx.forward_its = its
        return loss[0].clone()

    @staticmethod
    def backward(ctx, gout):
        prob, solver = ctx.prob, ctx.solver
        N, S, nc = prob["N"], prob["S"], prob["n_cells"]
        grad = _zeros(nc)
        scratch_loss = _zeros(1)
        Ub, Wb = {}, {}
        get = lambda d, k, n: d.setdefault(k, _zeros(n))
        adj_its = []
        for seg in sorted(ctx.ckpts, reverse=True):
            end = min(seg + ctx.ck, ctx.steps)
            st = _copy_state(ctx.ckpts[seg])
            states = [_copy_state(st)]
            for n in range(seg, end):
                api.time_step(solver, st, (n + 1) * prob["dt"], tol=ctx.tol)
                states.append(_copy_state(st))
            for n in reversed(range(seg, end)):
                cur, new = states[n - seg], states[n - seg + 1]
                ub = get(Ub, n + 1, N)
                api.sensor_misfit(solver, new.U, ctx.targets[n], ub, scratch_loss)
                lam = _zeros(N)
                r = api.pcg_solve(solver, ub, lam, tol=ctx.tol)
                adj_its.append(r["its"])
                api.grad_accumulate(solver, lam, new.U, grad)
                api.adjoint_step(solver, cur.U, cur.Uprev, cur.W, cur.Wprev, lam,
                                 get(Wb, n + 1, S * N), get(Ub, n, N), get(Ub, n - 1, N),
                                 get(Wb, n, S * N), get(Wb, n - 1, S * N))
                Ub.pop(n + 1, None)
                Wb.pop(n + 1, None)
        ctx.adjoint_its = adj_its
        return gout * grad, None, None, None, None, None, None


def sensor_misfit_loss(s, prob, targets, steps, tol=1e-13, checkpoint=10, precision="fp64"):
    """Differentiable sensor misfit of the time series at scalings s (cuda
    float64 tensor of length n_cells); targets: cuda tensor [steps, n_sensors]."""
    return SensorMisfit.apply(s, prob, targets, steps, tol, checkpoint, precision)
