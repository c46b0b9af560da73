"""Static condensation (HYB_STATIC) through the C ABI against the oracle.

The GPU assembles S = sum_T sigma-scattered S_hat_T with S_hat_T = L_bb
L_bb^T from the i-first element Cholesky; the oracle assembles
A_bb - A_bi A_ii^{-1} A_ib from dense solves (pinned against the Schur
complement of the conforming matrix).  Both are FP64 with different
rounding, each within 10 kappa_s 2^-53 of the exact values (kappa_s of the
equilibrated element matrices bounds that of their interior blocks), so
they agree to 20 kappa_s 2^-53 relative to the row (the observed value is
printed).  The solution through the GPU's
PCG and recovery equals the conforming solution (Theorem 2.1) and the
hybridized one.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import conforming
from oracle import static as ostat
from oracle import topology as otopo
from tests.gpu_common import kappa_of, norm_rel, oracle_gap_bound, rel_inf, require_gpu, row_rel_err

pytestmark = pytest.mark.gpu

CASES = [(0, 4, 0.2, True, False), (1, 3, 0.0, False, False), (1, 4, 0.2, True, True), (2, 3, 0.2, True, True),
         (3, 2, 0.2, True, False)]


def _problem(k, N, jit, rot, wg, seed):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=jit, rng=rng)
    if rot:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne, 0.5), synth.element_loads(rng, ne)
    g = rng.standard_normal((ne, 6 * (k + 1) ** 2)) if wg else None
    return mesh, a, b, f, g


def _plan(torch, mesh, k, a, b, f, g, system="static"):
    from paper_1801_08914_amd import Plan
    plan = Plan(mesh.xyz, mesh.e2v, k, system=system).bind()
    plan.setup(a, b, f, g)
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    return plan


@pytest.mark.parametrize("k,N,jit,rot,wg", CASES)
def test_S_and_load_match_oracle(k, N, jit, rot, wg):
    torch = require_gpu()
    print(f"case k={k} N={N} jitter={jit} rotate={rot} g={wg}", flush=True)
    mesh, a, b, f, g = _problem(k, N, jit, rot, wg, 7000 + 10 * k + N)
    plan = _plan(torch, mesh, k, a, b, f, g)
    ref = ostat.condense(k, mesh.xyz, mesh.e2v, a, b, f, g)
    rp, ci, val = [t.cpu().numpy() for t in plan.csr()]
    assert np.array_equal(ref.S.indptr, rp) and np.array_equal(ref.S.indices, ci)
    rg = plan.r().cpu().numpy()
    eS = row_rel_err(ref.S, val)
    er = rel_inf(ref.r, rg)
    bound = oracle_gap_bound(kappa_of(k, mesh, a, b, otopo.build_topology(mesh.e2v)))
    print(f"  S row-relative {eS:.1e}, normwise {norm_rel(ref.S.data, val):.1e}; load {er:.1e}; "
          f"bound 20 kappa_s u = {bound:.1e}", flush=True)
    assert eS <= bound and er <= bound


@pytest.mark.parametrize("k,N,jit,rot,wg", CASES)
def test_solution_equals_conforming_and_hybridized(k, N, jit, rot, wg):
    torch = require_gpu()
    mesh, a, b, f, g = _problem(k, N, jit, rot, wg, 7100 + 10 * k + N)
    ps = _plan(torch, mesh, k, a, b, f, g)
    x, info = ps.pcg(1e-13, 5000)
    assert info["converged"]
    u = ps.recover(x).cpu().numpy()
    ph = _plan(torch, mesh, k, a, b, f, g, system="hybrid")
    lam, ih = ph.pcg(1e-13, 5000)
    uh = ph.recover(lam).cpu().numpy()
    uc = conforming.conforming_solve(k, mesh.xyz, mesh.e2v, a, b, f, g)
    e1, e2 = rel_inf(uc, u), rel_inf(uh, u)
    print(f"k={k}: static u vs conforming {e1:.1e}, vs hybridized (GPU) {e2:.1e}; "
          f"PCG iterations S {info['iters']}, H {ih['iters']}", flush=True)
    assert e1 <= 1e-9 and e2 <= 1e-9


def test_static_rhs_reuse_and_argument_errors():
    torch = require_gpu()
    from paper_1801_08914_amd import HybError, Plan
    mesh, a, b, f, g = _problem(2, 3, 0.2, True, False, 7200)
    f2 = np.random.default_rng(3).standard_normal(f.shape)
    p1 = _plan(torch, mesh, 2, a, b, f, None)
    p1.rhs(f2)
    p2 = _plan(torch, mesh, 2, a, b, f2, None)
    torch.cuda.synchronize()
    assert torch.equal(p1.r().cpu(), p2.r().cpu())
    with pytest.raises(HybError):
        Plan(mesh.xyz, mesh.e2v, 2, system="static", precision="mixed")


def test_static_plans_in_a_batch_equal_single_plans():
    """Static-condensation plans of every order (with boundary data) in one
    batch, beside a hybridization plan: S, its load and the recovered u equal
    the single plans' bits, eager and on graph replays."""
    torch = require_gpu()
    from paper_1801_08914_amd import Batch, Plan
    cases = [(0, 4, "static"), (1, 3, "static"), (2, 3, "static"), (3, 2, "static"), (2, 2, "hybrid")]
    probs, plans, singles, xs = [], [], [], []
    for i, (k, N, system) in enumerate(cases):
        mesh, a, b, f, g = _problem(k, N, 0.2, True, True, 7300 + 10 * k + N)
        probs.append((mesh, k, a, b, f, g, system))
        plans.append(Plan(mesh.xyz, mesh.e2v, k, system=system, generic=True).bind())
        single = Plan(mesh.xyz, mesh.e2v, k, system=system, generic=True).bind()
        single.setup(a, b, f, g)
        x = np.random.default_rng(7400 + i).standard_normal(max(single.m, 1))
        u = single.recover(torch.as_tensor(x, device="cuda")).cpu()
        torch.cuda.synchronize()
        assert single.status()[0] == 0, (i, single.status())
        singles.append((single.csr()[2].cpu(), single.r().cpu(), u))
        xs.append(x)
    bt = Batch(plans)
    for i, (mesh, k, a, b, f, g, system) in enumerate(probs):
        bt.set(i, a, b, f, g=g, lam=xs[i])
    for graph in (False, True, True):
        bt.graph(graph)
        for pl in plans:
            pl.csr()[2].zero_()
            pl.r().zero_()
        bt.setup()
        bt.recover()
        torch.cuda.synchronize()
        for i, pl in enumerate(plans):
            assert pl.status()[0] == 0, (i, pl.status())
            assert torch.equal(pl.csr()[2].cpu(), singles[i][0]), (graph, i)
            assert torch.equal(pl.r().cpu(), singles[i][1]), (graph, i)
            assert torch.equal(bt.u(i).cpu(), singles[i][2]), (graph, i)
        print(f"  graph={graph}: {len(plans)} plans equal their single plans", flush=True)
