"""The boundary of the C ABI beyond the plain setup: natural boundary faces
(hyb_mesh.ess), the composite hyb_solve and hyb_get_csr, through the HIP
path against the oracle.

Natural boundary faces (Sec. 5 eliminates only the dofs whose normal flux is
prescribed): their dofs stay unknowns of the element and carry no multiplier.
H, r and u (for a seeded multiplier vector) are compared with the
long-double reference under the same bounds as the plain parity tests, with
prescribed fluxes g on the essential faces; the mixed-precision form and a
batch see the same faces.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import extended as oext
from oracle import hybrid as ohyb
from tests.gpu_common import (accuracy_bound, kappa_of, ld_dense, ld_row_errors, mixed_bound, norm_rel,
                              oracle_gap_bound, rel_inf, require_gpu)

pytestmark = pytest.mark.gpu

# (k, N, jitter, rotated frames)
CASES = [(0, 4, 0.2, True), (1, 3, 0.0, False), (1, 3, 0.2, True), (2, 3, 0.2, True), (3, 2, 0.2, False)]


def _problem(k, N, jit, rot, seed):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=jit, rng=rng)
    if rot:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne, 0.5), synth.element_loads(rng, ne)
    ess = rng.integers(0, 2, size=(ne, 6)).astype(np.uint8)      # about half the boundary faces natural
    g = rng.standard_normal((ne, 6 * (k + 1) ** 2))
    return mesh, a, b, f, ess, g


def _compare(plan, k, mesh, a, b, f, ess, g, bound):
    torch = require_gpu()
    ref = ohyb.hybridize(k, mesh.xyz, mesh.e2v, a, b, f, g_face=g, ess=ess)
    rp, ci, val = [t.cpu().numpy() for t in plan.csr()]
    assert np.array_equal(ref.H.indptr, rp) and np.array_equal(ref.H.indices, ci)
    rg = plan.r().cpu().numpy()
    els = np.arange(mesh.ne)
    lam = np.random.default_rng(5).standard_normal(plan.m)
    Hld, rld, U = oext.hybridize_ld(k, mesh.xyz, mesh.e2v, a, b, f, ref.topo, els, lam, ess=ess, g_face=g)
    Hg = sp.csr_matrix((val, ci, rp), shape=ref.H.shape)
    rows = np.arange(plan.m)
    eg, erg = ld_row_errors(Hld, rld, rows, Hg, rg)
    eo, ero = ld_row_errors(Hld, rld, rows, ref.H, ref.r)
    Hl, rl = ld_dense(Hld, rld, plan.m)
    ng, no = norm_rel(Hl, Hg.toarray()), norm_rel(Hl, ref.H.toarray())
    u = plan.recover(torch.as_tensor(lam, device="cuda")).cpu().numpy()
    uref = ohyb.recover(ref, mesh.xyz, mesh.e2v, a, b, f, lam, g_face=g)
    ul = np.array([U[e].astype(float) for e in els])
    eu, euo = rel_inf(ul, u), rel_inf(ul, uref)
    kap = kappa_of(k, mesh, a, b, ref.topo, ess=ess)
    print(f"  natural faces {int(((ess == 0) & (ref.topo.elem_face < 0)).sum())}: vs long double GPU / oracle "
          f"H {eg:.1e} / {eo:.1e} (normwise {ng:.1e} / {no:.1e}), r {erg:.1e} / {ero:.1e}, u {eu:.1e} / {euo:.1e}; "
          f"kappa_s {kap:.1e}", flush=True)
    assert eg <= bound(eo, kap) and erg <= bound(ero, kap) and ng <= bound(no, kap)
    assert eu <= bound(euo, kap)
    return ref, kap, val, rg, u


@pytest.mark.parametrize("k,N,jit,rot", CASES)
def test_natural_faces_fp64(k, N, jit, rot):
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    mesh, a, b, f, ess, g = _problem(k, N, jit, rot, 8100 + 10 * k + N)
    plan = Plan(mesh.xyz, mesh.e2v, k, ess=ess).bind()
    plan.setup(a, b, f, g)
    torch.cuda.synchronize()
    assert plan.status() == (0, -1)
    ref, kap, val, rg, _ = _compare(plan, k, mesh, a, b, f, ess, g, accuracy_bound)
    assert rel_inf(ref.H.data, val) <= oracle_gap_bound(kap) and rel_inf(ref.r, rg) <= oracle_gap_bound(kap)
    # every boundary face natural: no multiplier, the element blocks stay SPD
    plan2 = Plan(mesh.xyz, mesh.e2v, k, ess=np.zeros_like(ess)).bind()
    plan2.setup(a, b, f)
    torch.cuda.synchronize()
    assert plan2.status() == (0, -1)
    ref2 = ohyb.hybridize(k, mesh.xyz, mesh.e2v, a, b, f, ess=np.zeros_like(ess))
    kap2 = kappa_of(k, mesh, a, b, ref2.topo, ess=np.zeros_like(ess))
    assert rel_inf(ref2.H.data, plan2.csr()[2].cpu().numpy()) <= oracle_gap_bound(kap2)


@pytest.mark.parametrize("k,N,jit,rot", [c for c in CASES if c[0] in (1, 2)])
def test_natural_faces_mixed(k, N, jit, rot):
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    mesh, a, b, f, ess, g = _problem(k, N, jit, rot, 8200 + 10 * k + N)
    plan = Plan(mesh.xyz, mesh.e2v, k, ess=ess, precision="mixed").bind()
    plan.setup(a, b, f, g)
    torch.cuda.synchronize()
    assert plan.status() == (0, -1)
    _compare(plan, k, mesh, a, b, f, ess, g, mixed_bound)


def test_natural_faces_in_a_batch():
    """A batch holding plans with natural faces gives each plan's own bits."""
    torch = require_gpu()
    from paper_1801_08914_amd import Batch, Plan
    probs = [_problem(k, N, jit, rot, 8300 + i) for i, (k, N, jit, rot) in enumerate(CASES[:4])]
    singles, plans = [], []
    for (k, N, jit, rot), (mesh, a, b, f, ess, g) in zip(CASES[:4], probs):
        p = Plan(mesh.xyz, mesh.e2v, k, ess=ess, generic=True).bind()
        p.setup(a, b, f, g)
        lam = np.random.default_rng(3).standard_normal(max(p.m, 1))
        singles.append((p.csr()[2].clone(), p.r().clone(), p.recover(torch.as_tensor(lam[:p.m], device="cuda"))))
        plans.append(Plan(mesh.xyz, mesh.e2v, k, ess=ess, generic=True).bind())
    bt = Batch(plans)
    for i, (mesh, a, b, f, ess, g) in enumerate(probs):
        lam = np.random.default_rng(3).standard_normal(max(plans[i].m, 1))
        bt.set(i, a, b, f, g, lam=lam)
    bt.setup()
    bt.recover()
    torch.cuda.synchronize()
    for i, p in enumerate(plans):
        assert p.status() == (0, -1)
        H1, r1, u1 = singles[i]
        assert torch.equal(p.csr()[2], H1) and torch.equal(p.r(), r1) and torch.equal(bt.u(i), u1)


@pytest.mark.parametrize("k,precision", [(0, "fp64"), (1, "fp64"), (2, "fp64"), (1, "mixed"), (3, "fp64")])
def test_composite_solve_equals_its_steps(k, precision):
    """hyb_solve (rhs + PCG + recovery) gives the bits of the three calls, and
    hyb_get_csr points into the bound buffers."""
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    mesh, a, b, f, ess, g = _problem(k, 3 if k < 3 else 2, 0.2, True, 8400 + k)
    f2 = np.random.default_rng(11).standard_normal(f.shape)
    plan = Plan(mesh.xyz, mesh.e2v, k, ess=ess, precision=precision).bind()
    plan.setup(a, b, f, g)
    lam1, u1, info1 = plan.solve(f2, g, rtol=1e-13, maxit=5000)
    torch.cuda.synchronize()
    plan.rhs(f2, g)
    lam2, info2 = plan.pcg(1e-13, 5000)
    u2 = plan.recover(lam2)
    torch.cuda.synchronize()
    assert info1 == info2 and info1["converged"]
    assert torch.equal(lam1, lam2) and torch.equal(u1, u2)
    ptr = plan.csr_pointers()
    rp, ci, val = plan.csr()
    assert (ptr["row_ptr"], ptr["col"], ptr["val"]) == (rp.data_ptr(), ci.data_ptr(), val.data_ptr())
    assert (ptr["m"], ptr["nnz"]) == (plan.m, plan.nnz)
    # against the oracle's direct solve
    ref = ohyb.hybridize(k, mesh.xyz, mesh.e2v, a, b, f2, g_face=g, ess=ess)
    lref = ohyb.solve_reduced(ref.H, ref.r)
    uref = ohyb.recover(ref, mesh.xyz, mesh.e2v, a, b, f2, lref, g_face=g)
    eu = rel_inf(uref, u1.cpu().numpy())
    print(f"  k={k} {precision}: pcg {info1}, u vs oracle direct solve {eu:.1e}", flush=True)
    assert eu <= 1e-9
