"""The non-allocating PCG entry point (dgmg_pcg_solve_noalloc) against the
allocating one (dgmg_pcg_solve): the same solve, with the reduction scratch in
the library's static per-GPU array instead of the solver's buffers.

Two calls in a row through the C ABI, the second on a smaller problem (the
static array still holds the first call's partials and scalars): each result
must equal dgmg_pcg_solve's bit for bit (same kernels, same reduction order)
and match the oracle's direct solve."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from gpu_util import dev, host, need_gpu, rel, say, torch
from paper_2602_16312_amd import _ffi as F
from paper_2602_16312_amd import api, problem
from workloads import make_problem
from oracle.assemble import system_matrix

pytestmark = pytest.mark.gpu


def _call(entry, s, b, x0, tol, flexible):
    x = x0.clone()
    st = F.PCGStats()
    o = F.PCGOpts(tol, 0, 500, 1 if flexible else 0)
    torch.cuda.synchronize()
    rc = getattr(F.lib(), entry)(s.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                 C.byref(o), C.byref(st), None)
    torch.cuda.synchronize()
    return rc, st, x


# larger problem first, then a smaller one on the same static array
CASES = [("c2", 64, "mixed", False), ("c1", 16, "fp64", False), ("c1", 16, "fp64", True)]


def test_noalloc_pcg_matches_pcg_solve():
    need_gpu()
    for name, n, prec, flexible in CASES:
        pr = make_problem(name, n=n)
        A0, _, _, _ = system_matrix(pr)
        rng = np.random.default_rng(31 + n)
        b = A0 @ rng.standard_normal(pr["N"])
        x0 = rng.standard_normal(pr["N"]) * 0.1
        ref = sla.spsolve(A0.tocsc(), b)
        h, s = problem.build(pr, precision=prec)
        bd, x0d = dev(b), dev(x0)
        say("noalloc pcg", name, n, prec, "flexible" if flexible else "standard", "N", pr["N"])
        rc_a, st_a, x_a = _call("dgmg_pcg_solve_noalloc", s, bd, x0d, 1e-12, flexible)
        assert rc_a == 0, F.lib().dgmg_last_error()
        say("allocating pcg", name, n, prec)
        rc_b, st_b, x_b = _call("dgmg_pcg_solve", s, bd, x0d, 1e-12, flexible)
        assert rc_b == 0, F.lib().dgmg_last_error()
        assert (st_a.its, st_a.converged) == (st_b.its, st_b.converged)
        assert st_a.r0 == st_b.r0 and st_a.rfin == st_b.rfin
        assert torch.equal(x_a, x_b)
        assert rel(host(x_a), ref) <= 1e-10
        del s, h


def test_noalloc_pcg_zero_rhs_after_a_solve():
    """The array keeps the last call's contents: a zero right-hand side from a
    zero guess must still stop at once with a zero solution."""
    need_gpu()
    pr = make_problem("c1", n=16)
    h, s = problem.build(pr, precision="fp64")
    z = torch.zeros(pr["N"], dtype=torch.float64, device="cuda")
    say("noalloc pcg zero rhs")
    rc, st, x = _call("dgmg_pcg_solve_noalloc", s, z, z, 1e-10, False)
    assert rc == 0 and st.its == 0 and st.converged == 1 and st.r0 == 0.0
    assert float(x.abs().max()) == 0.0
