"""The M_s-weighted constraint of Example 2.3 through the C ABI: H' = M_s H
M_s and r' = M_s r against the oracle (M_s from face quadrature there, the
Gauss-weight closed form here; the long-double reference scaled by the same
diagonal), and the broken solution of the weighted system equal to the
unweighted one (lambda = M_s lambda')."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import extended as oext
from oracle import weighted as ow
from tests.gpu_common import accuracy_bound, kappa_of, ld_dense, norm_rel, oracle_gap_bound, rel_inf, require_gpu

pytestmark = pytest.mark.gpu

CASES = [(0, 4, 0.2, True), (1, 3, 0.0, False), (1, 3, 0.2, True), (2, 3, 0.2, True), (3, 2, 0.2, False)]


def _problem(k, N, jit, rot, seed):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=jit, rng=rng)
    if rot:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    return mesh, synth.lognormal(rng, ne), synth.lognormal(rng, ne, 0.5), synth.element_loads(rng, ne)


def _plan(torch, mesh, k, a, b, f, weighted):
    from paper_1801_08914_amd import Plan
    plan = Plan(mesh.xyz, mesh.e2v, k, weighted_c=weighted).bind()
    plan.setup(a, b, f)
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    return plan


@pytest.mark.parametrize("k,N,jit,rot", CASES)
def test_weighted_H_r_and_invariant_solution(k, N, jit, rot):
    torch = require_gpu()
    mesh, a, b, f = _problem(k, N, jit, rot, 8000 + 10 * k + N)
    pw = _plan(torch, mesh, k, a, b, f, True)
    Hw, rw, hy = ow.hybridize_weighted(k, mesh.xyz, mesh.e2v, a, b, f)
    rp, ci, val = [t.cpu().numpy() for t in pw.csr()]
    assert np.array_equal(Hw.indptr, rp) and np.array_equal(Hw.indices, ci)
    rg = pw.r().cpu().numpy()
    ms = ow.weights_vector(k, hy.r.size)
    if k < 3:
        Hld, rld, _ = oext.hybridize_ld(k, mesh.xyz, mesh.e2v, a, b, f, hy.topo, np.arange(mesh.ne))
        Hl, rl = ld_dense(Hld, rld, hy.r.size)
        Hl, rl = ms[:, None] * Hl * ms[None, :], ms * rl
        Hg = sp.csr_matrix((val, ci, rp), shape=Hw.shape).toarray()
        nH, nHo = norm_rel(Hl, Hg), norm_rel(Hl, Hw.toarray())
        nr, nro = norm_rel(rl, rg), norm_rel(rl, rw)
        kap = kappa_of(k, mesh, a, b, hy.topo)
        print(f"k={k}: weighted vs long double, GPU / oracle: H {nH:.1e} / {nHo:.1e}, r {nr:.1e} / {nro:.1e}; "
              f"kappa_s {kap:.1e}", flush=True)
        assert nH <= accuracy_bound(nHo, kap) and nr <= accuracy_bound(nro, kap)
    else:
        kap = kappa_of(k, mesh, a, b, hy.topo)
        e = norm_rel(Hw.data, val)
        print(f"k={k}: weighted H, GPU vs oracle {e:.1e}; kappa_s {kap:.1e}", flush=True)
        assert e <= oracle_gap_bound(kap)
    lw, iw = pw.pcg(1e-13, 5000)
    uw = pw.recover(lw).cpu().numpy()
    p0 = _plan(torch, mesh, k, a, b, f, False)
    l0, i0 = p0.pcg(1e-13, 5000)
    u0 = p0.recover(l0).cpu().numpy()
    e_lam = rel_inf(l0.cpu().numpy(), ms * lw.cpu().numpy())
    e_u = rel_inf(u0, uw)
    print(f"  lambda = M_s lambda' to {e_lam:.1e}, u weighted vs unweighted {e_u:.1e} "
          f"(PCG {iw['iters']} / {i0['iters']} iterations)", flush=True)
    assert iw["converged"] and e_lam <= 1e-9 and e_u <= 1e-10


def test_weighted_in_a_batch():
    """A batch of weighted plans equals the weighted plans' own calls."""
    torch = require_gpu()
    from paper_1801_08914_amd import Batch, Plan
    probs = [(_problem(k, 3, 0.2, True, 8100 + k), k) for k in (0, 1, 2)]
    plans = [Plan(m.xyz, m.e2v, k, weighted_c=True, generic=True).bind() for (m, a, b, f), k in probs]
    bt = Batch(plans)
    for i, ((m, a, b, f), k) in enumerate(probs):
        bt.set(i, a, b, f, lam=np.zeros(max(plans[i].m, 1)))
    bt.setup()
    torch.cuda.synchronize()
    for i, ((m, a, b, f), k) in enumerate(probs):
        single = _plan(torch, m, k, a, b, f, True)
        assert torch.equal(plans[i].csr()[2].cpu(), single.csr()[2].cpu())
        assert torch.equal(plans[i].r().cpu(), single.r().cpu())
