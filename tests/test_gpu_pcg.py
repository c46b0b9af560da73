"""Jacobi-PCG on the GPU (through the C ABI) against the oracle's PCG.

The GPU solver is handed the oracle's H and r (written into the plan's CSR
values and right-hand side), so both run the same iteration on the same
matrix and differ only by summation order inside the dot products and the
SpMV.  For a dot product of length m the two orders differ by at most
gamma_m = m 2^-53 relative to sum |x_i y_i|; after n iterations this compounds
to about n m 2^-53, which for the largest case here (m ~ 2.3e4, n <= 17) is
below 1e-10: the iterates after n steps must agree to 1e-10 normwise.  A full
solve (||r|| <= 1e-12 ||r_0||) must reach the direct solution to 1e-9 of its
largest entry, as the oracle's PCG does; the residual is looked at every 8
iterations, so the count is the oracle's count with the same checks, to within
one check period.  Row counts are not multiples of the 256 rows per block, and
the cases cover the 4-, 8- and 16-lanes-per-row SpMV.
"""
import numpy as np
import pytest

import synth
from oracle import hybrid as ohyb
from oracle.pcg import jacobi_pcg
from tests.gpu_common import norm_rel, require_gpu

pytestmark = pytest.mark.gpu

# (k, N, jitter, rotated frames): rows per SpMV row ~11 (k=0), 44 (k=1), 99 (k=2), 176 (k=3)
CASES = [(0, 8, 0.2, True), (1, 5, 0.2, False), (1, 12, 0.2, True), (2, 4, 0.2, True), (3, 3, 0.0, False)]


def _problem(k, N, jit, rot, seed):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=jit, rng=rng)
    if rot:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne, 0.5), synth.element_loads(rng, ne)
    return mesh, a, b, f


def _plan_with_oracle_system(torch, k, N, jit, rot, seed):
    from paper_1801_08914_amd import Plan
    mesh, a, b, f = _problem(k, N, jit, rot, seed)
    ref = ohyb.hybridize(k, mesh.xyz, mesh.e2v, a, b, f)
    plan = Plan(mesh.xyz, mesh.e2v, k).bind()
    plan.setup(a, b, f)
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    rp, ci, val = plan.csr()
    assert np.array_equal(rp.cpu().numpy(), ref.H.indptr) and np.array_equal(ci.cpu().numpy(), ref.H.indices)
    val.copy_(torch.as_tensor(ref.H.data, device=val.device))
    plan.r().copy_(torch.as_tensor(ref.r, device=val.device))
    print(f"k={k} N={N}: m={plan.m} nnz/row={plan.nnz / max(plan.m, 1):.1f}", flush=True)
    return plan, ref


@pytest.mark.parametrize("k,N,jit,rot", CASES)
def test_iterates_match_oracle_pcg(k, N, jit, rot):
    torch = require_gpu()
    plan, ref = _plan_with_oracle_system(torch, k, N, jit, rot, 700 + 10 * k + N)
    for n in (1, 2, 3, 8, 17):
        lam, info = plan.pcg(1e-30, n)
        assert info["iters"] == n and not info["converged"]
        lo, it, _, _ = jacobi_pcg(ref.H, ref.r, rtol=1e-30, maxit=n)
        assert it == n
        err = norm_rel(lo, lam.cpu().numpy())
        print(f"  after {n:2d} iterations: GPU vs oracle PCG {err:.1e}", flush=True)
        assert err <= 1e-10


@pytest.mark.parametrize("k,N,jit,rot", CASES)
def test_full_solve_matches_direct_solution(k, N, jit, rot):
    torch = require_gpu()
    plan, ref = _plan_with_oracle_system(torch, k, N, jit, rot, 800 + 10 * k + N)
    lam, info = plan.pcg(1e-12, 20000)
    lam = lam.cpu().numpy()
    direct = ohyb.solve_reduced(ref.H, ref.r)
    lo, it8, conv8, _ = jacobi_pcg(ref.H, ref.r, rtol=1e-12, maxit=20000, check_every=8)
    print(f"  GPU iters {info['iters']} (oracle {it8}), rel_res {info['rel_res']:.1e}, "
          f"vs direct {np.abs(lam - direct).max() / np.abs(direct).max():.1e}", flush=True)
    assert info["converged"] and conv8
    assert info["rel_res"] <= 1e-12
    assert abs(info["iters"] - it8) <= 8
    assert np.abs(lam - direct).max() <= 1e-9 * np.abs(direct).max()
    assert np.abs(lo - direct).max() <= 1e-9 * np.abs(direct).max()
    # deterministic: the same iterate bitwise on a second solve
    lam2, info2 = plan.pcg(1e-12, 20000)
    assert info2["iters"] == info["iters"] and np.array_equal(lam2.cpu().numpy(), lam)


@pytest.mark.parametrize("k,N", [(1, 6), (2, 4)])
def test_reduction_modes_agree_bitwise(k, N):
    """Partial sums inside the consuming kernels or in separate one-block
    kernels: the same partials in the same order, so the same bits."""
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    mesh, a, b, f = _problem(k, N, 0.2, True, 950 + k)
    out = []
    for mode in (1, 2):
        plan = Plan(mesh.xyz, mesh.e2v, k, pcg_reduce=mode).bind()
        plan.setup(a, b, f)
        lam, info = plan.pcg(1e-12, 5000)
        assert info["converged"]
        out.append((lam.cpu().numpy(), info["iters"], info["rel_res"]))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]


def test_not_converged_zero_rhs_and_empty_system():
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    plan, _ = _plan_with_oracle_system(torch, 1, 4, 0.2, False, 900)
    lam, info = plan.pcg(1e-14, 3)
    assert info["iters"] == 3 and not info["converged"] and info["rel_res"] > 1e-14
    plan.r().zero_()
    lam, info = plan.pcg(1e-12, 100)
    assert info["iters"] == 0 and info["converged"] and not lam.any()
    # one element: every face on the boundary, no multipliers
    mesh = synth.structured_hex(1)
    p1 = Plan(mesh.xyz, mesh.e2v, 1).bind()
    p1.setup(np.ones(1), np.ones(1), np.ones((1, 3)))
    assert p1.m == 0
    lam, info = p1.pcg(1e-12, 100)
    assert info["iters"] == 0 and info["converged"] and lam.numel() == 0
