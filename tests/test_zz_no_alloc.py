"""hyb_pcg_noalloc through the C ABI: the same iterates and bits as hyb_pcg
(whose work vectors live in the plan's bound work buffer), on two calls in a
row, the second with a smaller system, and a system too large for the
library's fixed array is refused with the bytes it would need."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu


def _plan(N, k, seed):
    from paper_1801_08914_amd import Plan
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=0.2, rng=rng)
    ne = mesh.ne
    plan = Plan(mesh.xyz, mesh.e2v, k).bind()
    plan.setup(synth.lognormal(rng, ne), synth.lognormal(rng, ne, 0.5), synth.element_loads(rng, ne))
    return plan


@pytest.mark.parametrize("k", [1, 2])
def test_noalloc_pcg_equals_pcg(k):
    torch = require_gpu()
    for N in (6, 3):                       # the second call on a smaller system
        plan = _plan(N, k, 900 + N)
        lam_a, info_a = plan.pcg(1e-12, 3000)
        torch.cuda.synchronize()
        lam_b, info_b = plan.pcg(1e-12, 3000, noalloc=True)
        torch.cuda.synchronize()
        print(f"k={k} N={N} m={plan.m}: {info_a} / {info_b}", flush=True)
        assert info_a == info_b and info_a["converged"]
        assert torch.equal(lam_a, lam_b)
        # a fixed iteration count that stops before convergence agrees too
        lam_c, info_c = plan.pcg(1e-30, 7)
        lam_d, info_d = plan.pcg(1e-30, 7, noalloc=True)
        torch.cuda.synchronize()
        assert info_c == info_d and info_c["iters"] == 7 and torch.equal(lam_c, lam_d)


def test_noalloc_refuses_a_system_beyond_its_array():
    torch = require_gpu()
    from paper_1801_08914_amd import Plan, _abi
    mesh = synth.structured_hex(48)
    plan = Plan(mesh.xyz, mesh.e2v, 1)             # m = 1,327,104 multipliers, host only
    lam = torch.empty(plan.m, dtype=torch.float64, device="cuda")
    info = _abi.HybSolveInfo()
    rc = plan._lib.hyb_pcg_noalloc(plan._plan, ctypes.c_double(1e-12), 10, ctypes.c_void_p(lam.data_ptr()),
                                   ctypes.byref(info))
    assert rc == _abi.HYB_E_ARG
    assert plan._lib.hyb_last_detail() > 48 * 2**20
