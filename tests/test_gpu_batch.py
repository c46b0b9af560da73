"""Uneven batches of problems of mixed order and mesh (through the C ABI; a
few launches per order and phase, mixed-precision problems in a persistent
launch): every problem's H, r and u equal those of its own plan calls
bitwise (same element routines), they match the oracle, hipGraph replays
equal the eager launches on every replay, and the autotuner's choice leaves
the results unchanged."""
import numpy as np
import pytest

import synth
import scipy.sparse as sp

from oracle import extended as oext
from oracle import hybrid as ohyb
from tests.gpu_common import accuracy_bound, kappa_of, ld_dense, norm_rel, oracle_gap_bound, require_gpu

pytestmark = pytest.mark.gpu


def _problems():
    # small C4-shaped batch: jittered n^3 meshes, n in 2..4, k in 0..3
    return synth.config_c4(nprob=8, nmin=2, nmax=4, seed=40)


def _batch(torch, probs):
    from paper_1801_08914_amd import Batch, Plan
    plans = [Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True).bind() for p in probs]
    b = Batch(plans)
    rng = np.random.default_rng(41)
    lams = [rng.standard_normal(max(pl.m, 1)) for pl in plans]
    for i, (p, pl) in enumerate(zip(probs, plans)):
        b.set(i, p.alpha, p.beta, p.f, lam=lams[i])
    return b, plans, lams


def _outputs(torch, b, plans):
    torch.cuda.synchronize()
    out = []
    for i, pl in enumerate(plans):
        rc, det = pl.status()
        assert rc == 0, (i, rc, det)
        out.append((pl.csr()[2].clone(), pl.r().clone(), b.u(i).clone()))
    return out


def test_batch_matches_single_plans_and_oracle():
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    probs = _problems()
    print("orders", [p.k for p in probs], "elements", [p.mesh.ne for p in probs], flush=True)
    assert sorted(set(p.k for p in probs)) == [0, 1, 2, 3]
    b, plans, lams = _batch(torch, probs)
    b.setup()
    b.recover()
    got = _outputs(torch, b, plans)
    for i, p in enumerate(probs):
        single = Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True).bind()
        single.setup(p.alpha, p.beta, p.f)
        u = single.recover(torch.as_tensor(lams[i], device="cuda")).cpu()
        torch.cuda.synchronize()
        val, r, ub = got[i]
        assert torch.equal(val.cpu(), single.csr()[2].cpu()), i
        assert torch.equal(r.cpu(), single.r().cpu()), i
        assert torch.equal(ub.cpu(), u), i
        # and against the long-double reference: at least as accurate as the
        # FP64 oracle (normwise; the per-entry form is exercised by the
        # single-plan parity tests)
        args = (p.k, p.mesh.xyz, p.mesh.e2v, p.alpha, p.beta, p.f)
        ref = ohyb.hybridize(*args)
        Hld, rld, U = oext.hybridize_ld(*args, ref.topo, np.arange(p.mesh.ne), lams[i][:ref.r.size])
        Hl, rl = ld_dense(Hld, rld, ref.r.size)
        Hg = sp.csr_matrix((val.cpu().numpy(), ref.H.indices, ref.H.indptr), shape=ref.H.shape).toarray()
        ul = np.array([U[e].astype(float) for e in range(p.mesh.ne)])
        uref = ohyb.recover(ref, p.mesh.xyz, p.mesh.e2v, p.alpha, p.beta, p.f, lams[i][:ref.r.size])
        eH, eHo = norm_rel(Hl, Hg), norm_rel(Hl, ref.H.toarray())
        er, ero = norm_rel(rl, r.cpu().numpy()), norm_rel(rl, ref.r)
        eu, euo = norm_rel(ul, ub.cpu().numpy()), norm_rel(ul, uref)
        kap = kappa_of(p.k, p.mesh, p.alpha, p.beta, ref.topo)
        print(f"  problem {i} k={p.k} ne={p.mesh.ne}: vs long double, GPU / oracle: H {eH:.1e} / {eHo:.1e} "
              f"r {er:.1e} / {ero:.1e} u {eu:.1e} / {euo:.1e}; kappa_s {kap:.1e}", flush=True)
        assert eH <= accuracy_bound(eHo, kap) and er <= accuracy_bound(ero, kap) and eu <= accuracy_bound(euo, kap)
        assert norm_rel(ref.H.toarray(), Hg) <= oracle_gap_bound(kap)
        assert norm_rel(uref, ub.cpu().numpy()) <= oracle_gap_bound(kap)


def test_batch_graph_replays_and_autotune():
    torch = require_gpu()
    probs = _problems()
    b, plans, _ = _batch(torch, probs)
    b.setup()
    b.recover()
    eager = _outputs(torch, b, plans)
    b.graph(True)
    for rep in range(3):
        # eager work of the program between replays
        torch.empty(1 << 20, dtype=torch.float64, device="cuda").fill_(float(rep))
        for pl in plans:
            pl.csr()[2].zero_()
            pl.r().zero_()
        b.setup()
        b.recover()
        out = _outputs(torch, b, plans)
        for i in range(len(plans)):
            assert all(torch.equal(x, y) for x, y in zip(eager[i], out[i])), (rep, i)
    b.graph(False)
    best = b.autotune(reps=1)
    print("autotuned tiles", best, flush=True)
    assert b.tiles() == best
    b.setup()
    b.recover()
    tuned = _outputs(torch, b, plans)
    for i in range(len(plans)):
        assert all(torch.equal(x, y) for x, y in zip(eager[i], tuned[i])), i


def test_batch_padding_teams_leave_rt3_records_alone():
    """RT3 recovers eight elements per workgroup (one per wave), RT2 two:
    past a problem's last element the padding teams take element 0 as their
    safe index and must write nothing.  One- and 27-element RT3 problems
    (and an RT2 one between them) give the single plans' bits."""
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    rng = np.random.default_rng(45)
    probs = []
    for n, k in ((1, 3), (3, 2), (3, 3)):
        mesh = synth.structured_hex(n, jitter=0.2 if n > 1 else 0.0, rng=rng)
        probs.append(synth.Problem(f"pad_k{k}_n{n}", mesh, k, synth.lognormal(rng, mesh.ne),
                                   synth.lognormal(rng, mesh.ne, 0.5), synth.element_loads(rng, mesh.ne)))
    b, plans, lams = _batch(torch, probs)
    for rep in range(2):
        b.setup()
        b.recover()
        got = _outputs(torch, b, plans)
        for i, p in enumerate(probs):
            single = Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True).bind()
            single.setup(p.alpha, p.beta, p.f)
            u = single.recover(torch.as_tensor(lams[i], device="cuda")).cpu()
            torch.cuda.synchronize()
            assert single.status()[0] == 0
            val, r, ub = got[i]
            print(f"  replay {rep} problem {i} k={p.k} ne={p.mesh.ne}", flush=True)
            assert torch.equal(val.cpu(), single.csr()[2].cpu()), i
            assert torch.equal(r.cpu(), single.r().cpu()), i
            assert torch.equal(ub.cpu(), u), i


def test_batch_more_problems_per_order_than_one_launch_takes():
    """RT2 and RT3 problems go eight to a launch (their descriptors in the
    kernel arguments): ten RT3 and nine RT2 problems of 1 or 8 elements, and
    two RT1 ones, take several launches per order and phase; every problem
    gives its single plan's bits, eager and on graph replays."""
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    rng = np.random.default_rng(49)
    probs = []
    for i, (n, k) in enumerate([(1 + (i % 2), 3) for i in range(10)] + [(2 - (i % 2), 2) for i in range(9)] +
                               [(2, 1), (1, 1)]):
        mesh = synth.structured_hex(n, jitter=0.2 if n > 1 else 0.0, rng=rng)
        probs.append(synth.Problem(f"many_{i}_k{k}_n{n}", mesh, k, synth.lognormal(rng, mesh.ne),
                                   synth.lognormal(rng, mesh.ne, 0.5), synth.element_loads(rng, mesh.ne)))
    b, plans, lams = _batch(torch, probs)
    singles = []
    for i, p in enumerate(probs):
        single = Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True).bind()
        single.setup(p.alpha, p.beta, p.f)
        u = single.recover(torch.as_tensor(lams[i], device="cuda")).cpu()
        torch.cuda.synchronize()
        assert single.status()[0] == 0, (i, single.status())
        singles.append((single.csr()[2].cpu(), single.r().cpu(), u))
    for graph in (False, True, True):
        b.graph(graph)
        for pl in plans:
            pl.csr()[2].zero_()
            pl.r().zero_()
        b.setup()
        b.recover()
        got = _outputs(torch, b, plans)
        for i, p in enumerate(probs):
            val, r, ub = got[i]
            assert torch.equal(val.cpu(), singles[i][0]), (graph, i, p.name)
            assert torch.equal(r.cpu(), singles[i][1]), (graph, i, p.name)
            assert torch.equal(ub.cpu(), singles[i][2]), (graph, i, p.name)
        print(f"  graph={graph}: {len(probs)} problems equal their single plans", flush=True)


def test_batch_mixed_and_fp64_plans_together():
    """A batch of FP64 and mixed-precision (HYB_MIXED) problems of every
    order: the mixed problems run in their own persistent launch per phase;
    every problem gives its single plan's bits, on eager launches and on
    every graph replay, and the mixed ones stay within the refined bound of
    the oracle's solution."""
    torch = require_gpu()
    from paper_1801_08914_amd import Batch, Plan
    probs = synth.config_c4(nprob=8, nmin=2, nmax=3, seed=47)
    ks = [p.k for p in probs]
    print("orders", ks, "elements", [p.mesh.ne for p in probs], flush=True)
    assert sorted(set(ks)) == [0, 1, 2, 3]
    # per order: the first problem mixed, the rest FP64
    mixed = [ks.index(k) == i for i, k in enumerate(ks)]
    prec = ["mixed" if mx else "fp64" for mx in mixed]
    plans = [Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True, precision=pc).bind() for p, pc in zip(probs, prec)]
    b = Batch(plans)
    rng = np.random.default_rng(48)
    lams = [rng.standard_normal(max(pl.m, 1)) for pl in plans]
    for i, p in enumerate(probs):
        b.set(i, p.alpha, p.beta, p.f, lam=lams[i])
    singles = []
    for i, p in enumerate(probs):
        single = Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True, precision=prec[i]).bind()
        single.setup(p.alpha, p.beta, p.f)
        u = single.recover(torch.as_tensor(lams[i], device="cuda")).cpu()
        torch.cuda.synchronize()
        assert single.status()[0] == 0, (i, single.status())
        singles.append((single.csr()[2].cpu(), single.r().cpu(), u))
    for graph in (False, True, True):
        b.graph(graph)
        b.setup()
        b.recover()
        got = _outputs(torch, b, plans)
        for i in range(len(probs)):
            val, r, ub = got[i]
            print(f"  graph={graph} problem {i} k={ks[i]} {prec[i]}", flush=True)
            assert torch.equal(val.cpu(), singles[i][0]), i
            assert torch.equal(r.cpu(), singles[i][1]), i
            assert torch.equal(ub.cpu(), singles[i][2]), i
        torch.cuda.synchronize()
    for i, p in enumerate(probs):
        if not mixed[i]:
            continue
        args = (p.k, p.mesh.xyz, p.mesh.e2v, p.alpha, p.beta, p.f)
        ref = ohyb.hybridize(*args)
        Hg = sp.csr_matrix((singles[i][0].numpy(), ref.H.indices, ref.H.indptr), shape=ref.H.shape)
        eH = norm_rel(ref.H.toarray(), Hg.toarray())
        er = norm_rel(ref.r, singles[i][1].numpy())
        print(f"  mixed problem {i} k={p.k}: H {eH:.1e} r {er:.1e} vs the FP64 oracle", flush=True)
        assert max(eH, er) <= 1e-10


def test_batch_mixed_results_do_not_depend_on_tiles():
    """All-mixed batch of every order: the refinement ends at different
    sweeps in different teams of a block, and persistent blocks go on from
    one order's items to another's (another LDS layout); H and r are the same
    bits whatever the grid and items per block."""
    torch = require_gpu()
    from paper_1801_08914_amd import Batch, Plan
    probs = synth.config_c4(nprob=10, nmin=3, nmax=6, seed=50)
    assert sorted(set(p.k for p in probs)) == [0, 1, 2, 3]
    outs = []
    for tiles in ((1, 1), (8, 1), (2, 4)):
        plans = [Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True, precision="mixed").bind() for p in probs]
        b = Batch(plans)
        for i, p in enumerate(probs):
            b.set(i, p.alpha, p.beta, p.f)
        b.tiles(*tiles)
        b.setup()
        torch.cuda.synchronize()
        outs.append([(pl.csr()[2].cpu(), pl.r().cpu(), pl.status()[0]) for pl in plans])
        print(f"  tiles {tiles}: statuses {[o[2] for o in outs[-1]]}", flush=True)
    for o in outs[1:]:
        for i in range(len(probs)):
            assert o[i][2] == outs[0][i][2], i
            assert torch.equal(o[i][0], outs[0][i][0]), i
            assert torch.equal(o[i][1], outs[0][i][1]), i


def test_affine_rt1_plan_switched_by_a_batch():
    """An affine RT_1 plan set up by its own (affine-specific) kernels and
    then put in a batch: its factors are in the other kernels' layout, so
    rhs / recover are refused until the batch (or hyb_setup) has set it up
    again; after the batch setup its recovery equals a generic single plan."""
    torch = require_gpu()
    from paper_1801_08914_amd import Batch, HybError, Plan, _abi
    rng = np.random.default_rng(44)
    mesh = synth.structured_hex(3)
    a, b, f = synth.lognormal(rng, mesh.ne), synth.lognormal(rng, mesh.ne), synth.element_loads(rng, mesh.ne)
    plan = Plan(mesh.xyz, mesh.e2v, 1).bind()
    plan.setup(a, b, f)
    lam = rng.standard_normal(plan.m)
    bt = Batch([plan])
    with pytest.raises(HybError) as ei:
        plan.recover(lam)
    assert ei.value.code == _abi.HYB_E_STATE
    bt.set(0, a, b, f, lam=lam)
    bt.setup()
    u = plan.recover(torch.as_tensor(lam, device="cuda")).cpu()
    single = Plan(mesh.xyz, mesh.e2v, 1, generic=True).bind()
    single.setup(a, b, f)
    u1 = single.recover(torch.as_tensor(lam, device="cuda")).cpu()
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    assert torch.equal(u, u1)
    assert torch.equal(plan.csr()[2].cpu(), single.csr()[2].cpu())
