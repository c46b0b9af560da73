"""Serving loop: requests admitted by slots and device-memory budget run
overlapped on their own streams; every result is the same (bitwise) alone
and in the mix, and matches the oracle's solve."""
import numpy as np
import pytest

import synth
from oracle import hybrid as ohyb
from tests.gpu_common import rel_inf, require_gpu

pytestmark = pytest.mark.gpu


def _requests():
    # small requests shaped like the serving stream: jittered meshes, k in
    # 1..3, 1..3 right-hand sides reusing the factors
    from paper_1801_08914_amd.serving import Request
    out = []
    for t, prob, fs in synth.serving_requests(6, qps=1000.0, seed=50, nmin=2, nmax=3, rmax=3):
        out.append((t, Request(prob.mesh.xyz, prob.mesh.e2v, prob.k, prob.alpha, prob.beta, fs, tag=prob.name)))
    return out


def _run(slots, budget, reqs, together):
    from paper_1801_08914_amd.serving import Server
    srv = Server(budget, slots=slots, rtol=1e-13)
    try:
        if together:
            futs = [srv.submit(r) for _, r in reqs]
            return [f.result(timeout=240) for f in futs]
        return [srv.submit(r).result(timeout=240) for _, r in reqs]
    finally:
        srv.close()


def test_results_same_alone_and_in_the_mix():
    require_gpu()
    reqs = _requests()
    print("requests", [(r.k, r.xyz.shape[0], len(r.loads)) for _, r in reqs], flush=True)
    alone = _run(1, 1 << 40, reqs, together=False)
    mix = _run(4, 1 << 40, reqs, together=True)
    # in the mix, requests overlapped in time
    spans = sorted((r.admitted, r.done) for r in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for a, b in zip(alone, mix):
        assert a.tag == b.tag and len(a.u) == len(b.u)
        for ua, ub in zip(a.u, b.u):
            assert np.array_equal(ua, ub), a.tag
        assert a.converged and b.converged
    # against the oracle's direct solve, every load of every request
    for (_, r), res in zip(reqs, mix):
        for f, u in zip(r.loads, res.u):
            ref = ohyb.hybridize(r.k, r.xyz, r.e2v, r.alpha, r.beta, f)
            lam = ohyb.solve_reduced(ref.H, ref.r)
            uref = ohyb.recover(ref, r.xyz, r.e2v, r.alpha, r.beta, f, lam)
            err = rel_inf(uref, u)
            print(f"  {r.k} {res.tag}: u vs oracle {err:.1e}", flush=True)
            assert err <= 1e-9


def test_admission_by_memory_budget():
    require_gpu()
    from paper_1801_08914_amd import Plan
    from paper_1801_08914_amd.serving import footprint_bytes
    reqs = _requests()
    needs = [footprint_bytes(Plan(r.xyz, r.e2v, r.k).sizes) for _, r in reqs]
    # room for the largest request only: whatever runs at the same time fits
    budget = max(needs)
    res = _run(4, budget, reqs, together=True)
    for r in res:
        running = sum(q.footprint for q in res if q.admitted <= r.admitted < q.done)
        assert running <= budget
    alone = _run(1, 1 << 40, reqs, together=False)
    for a, b in zip(alone, res):
        for ua, ub in zip(a.u, b.u):
            assert np.array_equal(ua, ub)
    # a request larger than the whole budget is refused
    from paper_1801_08914_amd.serving import Server
    srv = Server(min(needs) - 1, slots=2)
    try:
        with pytest.raises(MemoryError):
            srv.submit(reqs[0][1]).result(timeout=60)
    finally:
        srv.close()


def test_a_failing_request_leaves_the_others_unchanged():
    """One request in the mix has an indefinite element matrix (negative mass
    coefficient on one element): it fails with HYB_E_NOT_SPD and that
    element, the requests around it complete with the bits they have alone."""
    require_gpu()
    import dataclasses

    from paper_1801_08914_amd import _abi
    from paper_1801_08914_amd.serving import Server
    reqs = _requests()
    bad_at = 2
    _, r = reqs[bad_at]
    alpha = r.alpha.copy()
    alpha[1] = -5.0
    bad = dataclasses.replace(r, alpha=alpha, beta=r.beta * 1e-3, tag="bad")
    good = [q for i, (_, q) in enumerate(reqs) if i != bad_at]
    alone = _run(1, 1 << 40, [(0.0, q) for q in good], together=False)
    srv = Server(1 << 40, slots=4, rtol=1e-13)
    try:
        order = good[:bad_at] + [bad] + good[bad_at:]
        futs = [srv.submit(q) for q in order]
        out = []
        for q, fu in zip(order, futs):
            if q.tag == "bad":
                with pytest.raises(RuntimeError) as ei:
                    fu.result(timeout=240)
                assert f"device error {_abi.HYB_E_NOT_SPD} at element 1" in str(ei.value)
            else:
                out.append(fu.result(timeout=240))
    finally:
        srv.close()
    for a, b in zip(alone, out):
        assert a.tag == b.tag
        for ua, ub in zip(a.u, b.u):
            assert np.array_equal(ua, ub), a.tag
