"""Device memory through the caller's allocator (torch's caching allocator):
every solver buffer and set-up temporary comes from it and goes back to it,
results are bitwise identical to the library's own allocations, and a failing
allocator is reported as DGMG_ENOMEM."""
import numpy as np
import pytest

from gpu_util import dev, host, need_gpu, say, torch
from paper_2602_16312_amd import api, problem
from paper_2602_16312_amd import _ffi as F
from paper_2602_16312_amd._ffi import DGMGError
from workloads import make_problem
from workloads.configs import iapp_nodal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _steps(pr, s, n):
    N = pr["N"]
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(N, dtype=torch.float64, device="cuda"))
    its = []
    for k in range(n):
        t = (k + 1) * pr["dt"]
        r = api.time_step(s, st, t, iapp=dev(iapp_nodal(pr, t)), tol=1e-10)
        assert r["converged"]
        its.append(r["its"])
    return its, host(st.U)


@pytest.mark.parametrize("setup", ["host", "device"])
def test_torch_allocator_matches_own_allocations(setup):
    pr = make_problem("c2", n=16)
    say("allocator reference", setup)
    h1, s1 = problem.build(pr, precision="mixed", setup=setup)
    its1, U1 = _steps(pr, s1, 3)
    alloc = api.TorchAllocator()
    say("allocator torch", setup)
    h2, s2 = problem.build(pr, precision="mixed", setup=setup, allocator=alloc)
    # after set-up only the solver's own buffers are held (temporaries returned)
    assert alloc.live_bytes >= s2.info()["device_bytes"]
    assert alloc.live_bytes <= s2.info()["device_bytes"] + 256 * len(alloc.live)
    its2, U2 = _steps(pr, s2, 3)
    assert its1 == its2
    assert np.array_equal(U1, U2)
    del s2
    assert alloc.live == {}


def test_failing_allocator_reports_enomem():
    class Failing(api.TorchAllocator):
        def __init__(self):
            super().__init__()
            self._c_alloc = F.ALLOC_FN(lambda ctx, n: None)
            self.struct = F.Allocator(self._c_alloc, self._c_free, None)

    pr = make_problem("c1", n=8)
    alloc = Failing()
    say("failing allocator")
    with pytest.raises(DGMGError) as e:
        problem.build(pr, setup="device", allocator=alloc)
    assert e.value.code == -5   # DGMG_ENOMEM
    assert alloc.live == {}
