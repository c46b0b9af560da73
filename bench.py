"""Throughput of the hybridization hot path on one MI355X.

One step = the whole path for one batch of elements: per-element assembly of
M_T and f_T, Cholesky, H_T and its scatter into CSR H, r (setup), then the
element-by-element recovery of u from lambda.  The Jacobi-PCG that produces
lambda runs once before the timed region and is reported separately.

Prints one JSON line: the value, a roofline object for the dominant kernel
and the oracle timed on the host cores as a reported baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hybridized elements/s (setup+recover) vs FP64 plain at stated error; p50/p99 lat"
HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP64_PEAK = 78.6e12        # flop/s, MI355X FP64 (vector = matrix)


def per_element_counts(k: int, ne: int, nnz: int, m: int, nv: int):
    """Algorithmic bytes and flops per element of the setup (with the
    right-hand side) and of the recovery.

    Bytes: inputs (vertex ids and coordinates, alpha, beta, f, the element's
    face data), the factor record (interior inverse, E = A_ii^-1 A_ib and
    S^-1: n(n+1)/2 doubles for every order), y, the element's share of the CSR
    values of H and of r.  Flops: assembly (4 per entry of M_T) and the
    Gauss-Jordan condensation as the kernels do it: every interior pivot
    updates the n x (n+1) augmented matrix, every face pivot the
    nb x (nb+1) face block."""
    K2 = (k + 1) ** 2
    n = 3 * K2 * (k + 2)
    nb = 6 * K2
    ni = n - nb
    npk = n * (n + 1) // 2
    inputs = 8 * 4 + 24.0 * nv / ne + 8 + 8 + 24 + 6 * 4 + 8 + 36   # e2v, coords, alpha, beta, f, maps
    setup_bytes = inputs + 8 * npk + 8 * n + 8.0 * nnz / ne + 8.0 * m / ne
    setup_flops = 4 * n * n + 2 * ni * n * (n + 1) + 2 * nb * nb * (nb + 1)
    rec_bytes = 8 * (npk - ni * (ni + 1) // 2) + 8 * n + 8 * nb + 8 * n + 6 * 4 + 8
    rec_flops = 2 * nb * nb + 2 * ni * nb
    return dict(setup_bytes=setup_bytes, setup_flops=setup_flops, recover_bytes=rec_bytes, recover_flops=rec_flops)


def algo_counts(k: int):
    """Algorithmic count per element of order k, the work the method itself
    must do (the dense weighted Gram assembly 2 n^2 Q, the Cholesky n^3/3,
    the inverse of the face block 2 nb^3/3) and the bytes of the recovery
    (the generic factor record read, y, the element's multipliers, u
    written)."""
    K2 = (k + 1) ** 2
    n, nb, Q = 3 * K2 * (k + 2), 6 * K2, (k + 2) ** 3
    flops = 2 * n * n * Q + n ** 3 / 3 + 2 * nb ** 3 / 3
    rec_bytes = 8 * (n * (n + 1) // 2 + 2 * n + nb) + 6 * 4 + 8
    return dict(setup_flops=flops, recover_bytes=rec_bytes)


def host_cpu():
    """Model name and logical CPU count of the host (for cpu_baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def _sum_or_none(*xs):
    return None if any(x is None for x in xs) else float(sum(xs))


def traffic_from_profile(kernel: str, ne: int, fname: str = "hbm_traffic_rt1_32cubed.json"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain device copy), or None
    when the summary is missing or the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("sources_sha256") or rec.get("elements") != ne:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def cpu_baseline(prob, target_s: float = 12.0):
    """The oracle as it stands, single-threaded BLAS, on a bounded sample of
    the same workload: setup (with rhs) + recovery of the first S elements."""
    from threadpoolctl import threadpool_limits

    from oracle import hybrid as ohyb
    from oracle import topology as otopo
    topo = otopo.build_topology(prob.mesh.e2v)
    mid, _ = otopo.multiplier_map(topo, prob.k)
    m = topo.nfaces * (prob.k + 1) ** 2
    lam = np.random.default_rng(0).standard_normal(m)
    args = (prob.k, prob.mesh.xyz, prob.mesh.e2v, prob.alpha, prob.beta, prob.f)

    def run(S):
        els = np.arange(S)
        t0 = time.perf_counter()
        hyb = ohyb.hybridize(*args, topo=topo, elements=els, mult_id=mid)
        ohyb.recover(hyb, prob.mesh.xyz, prob.mesh.e2v, prob.alpha, prob.beta, prob.f, lam, elements=els)
        return time.perf_counter() - t0

    with threadpool_limits(1):
        S = min(256, prob.mesh.ne)
        t = run(S)
        S = int(min(prob.mesh.ne, max(S, S * target_s / max(t, 1e-3))))
        t = run(S)
    return {"value": S / t, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"first {S} of {prob.mesh.ne} elements of the same workload, setup incl. rhs + recovery, "
                      f"{t:.1f} s, 1 thread (BLAS limited to 1)"}


_MIX = []   # (problem, topology, multiplier ids) of the CPU baseline, inherited by forked workers


def _oracle_chunk(args):
    """Worker: _oracle_task on problem i of _MIX, elements [e0, e1)."""
    i, e0, e1 = args
    p, topo, mid = _MIX[i]
    return _oracle_task((p.k, p.mesh.xyz, p.mesh.e2v, p.alpha, p.beta, p.f, topo, mid, e0, e1, i))


def _oracle_task(args):
    """One oracle run: setup with rhs + recovery of the elements [e0, e1) of
    one problem; returns (elements, seconds)."""
    k, xyz, e2v, alpha, beta, f, topo, mid, e0, e1, seed = args
    from threadpoolctl import threadpool_limits

    from oracle import hybrid as ohyb
    with threadpool_limits(1):
        lam = np.random.default_rng(seed).standard_normal(topo.nfaces * (k + 1) ** 2)
        els = np.arange(e0, e1)
        t0 = time.perf_counter()
        hyb = ohyb.hybridize(k, xyz, e2v, alpha, beta, f, topo=topo, elements=els, mult_id=mid)
        ohyb.recover(hyb, xyz, e2v, alpha, beta, f, lam, elements=els)
        return e1 - e0, time.perf_counter() - t0


def cpu_baseline_mix(probs, target_s: float = 12.0, label: str = "the same workload"):
    """The oracle as it stands on a bounded sample of a multi-problem
    workload: the same fraction of every problem's elements (so the order
    mix is the workload's), setup with rhs + recovery, single-threaded BLAS
    per process; once in one process and once over min(usable CPUs, 16)
    processes.  Run before the GPU is initialised: the workers are forked
    and inherit the inputs."""
    import multiprocessing as mp

    from oracle import topology as otopo
    model, ncpu, usable = host_cpu()
    # topology and multiplier numbering once per problem (host planning, not timed)
    topos = []
    for p in probs:
        topo = otopo.build_topology(p.mesh.e2v)
        topos.append((topo, otopo.multiplier_map(topo, p.k)[0]))
    # per-order oracle cost from a small probe in this process
    per_k = {}
    for p, (topo, mid) in zip(probs, topos):
        if p.k not in per_k:
            s = min(4, p.mesh.ne)
            _, t = _oracle_task((p.k, p.mesh.xyz, p.mesh.e2v, p.alpha, p.beta, p.f, topo, mid, 0, s, 0))
            per_k[p.k] = t / s
    est = sum(per_k[p.k] * p.mesh.ne for p in probs)
    frac = min(1.0, target_s / max(est, 1e-9))
    tasks = []
    for i, (p, (topo, mid)) in enumerate(zip(probs, topos)):
        s = max(1, int(round(frac * p.mesh.ne)))
        tasks.append((p.k, p.mesh.xyz, p.mesh.e2v, p.alpha, p.beta, p.f, topo, mid, 0, s, i))
    out = {"unit": "elements/s", "kind": "oracle", "cpu_model": model, "logical_cpus": ncpu,
           "usable_cpus": usable}
    res = [_oracle_task(t) for t in tasks]
    nel, t1 = sum(r[0] for r in res), sum(r[1] for r in res)
    out["value"] = nel / t1
    out["cores"] = 1
    out["sample"] = (f"{frac:.3%} of every problem's elements ({nel} of {sum(p.mesh.ne for p in probs)}) of "
                     f"{label}, setup incl. rhs + recovery (topology not timed), {t1:.1f} s, 1 process, "
                     f"BLAS limited to 1 thread")
    procs = max(1, min(usable, 16))
    # every problem's sample in chunks of about equal cost, largest first
    chunks = []
    for i, t in enumerate(tasks):
        k, e0, e1 = t[0], t[8], t[9]
        step = 1 if k == 3 else max(1, (e1 - e0 + 3) // 4)
        for c0 in range(e0, e1, step):
            chunks.append((per_k[k] * (min(e1, c0 + step) - c0), (i, c0, min(e1, c0 + step))))
    chunks = [c for _, c in sorted(chunks, key=lambda x: -x[0])]
    _MIX[:] = [(p, topo, mid) for p, (topo, mid) in zip(probs, topos)]
    ctx = mp.get_context("fork")
    with ctx.Pool(processes=procs) as pool:
        pool.map(_oracle_chunk, [(0, 0, 1)] * procs)    # warm the workers
        t0 = time.perf_counter()
        resp = pool.map(_oracle_chunk, chunks, chunksize=1)
        tp = time.perf_counter() - t0
    _MIX.clear()
    out["multi_process"] = {"value": sum(r[0] for r in resp) / tp, "cores": procs, "seconds": tp,
                            "sample": "the same sample in chunks over a process pool (forked workers, "
                                      "1 BLAS thread each); wall time of the pool"}
    return out


def parity_sample(prob, plan, lam_np, nface=48, nel=48, seed=0):
    """Error of the GPU H rows, r and u against the oracle on sampled faces
    and elements (both elements of a sampled face are computed, so its rows
    of H are complete)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg  # noqa: F401  (sp.linalg.norm)

    from oracle import hybrid as ohyb
    from oracle import topology as otopo
    rng = np.random.default_rng(seed)
    topo = otopo.build_topology(prob.mesh.e2v)
    faces = rng.choice(topo.nfaces, size=min(nface, topo.nfaces), replace=False)
    els = np.unique(np.concatenate([topo.face_owner[faces, 0], topo.face_nbr[faces, 0],
                                    rng.choice(prob.mesh.ne, size=min(nel, prob.mesh.ne), replace=False)]))
    args = (prob.k, prob.mesh.xyz, prob.mesh.e2v, prob.alpha, prob.beta, prob.f)
    ref = ohyb.hybridize(*args, topo=topo, elements=els)
    rp, ci, val = [t.cpu().numpy() for t in plan.csr()]
    Hg = sp.csr_matrix((val, ci, rp), shape=(plan.m, plan.m))
    K2 = (prob.k + 1) ** 2
    eH = er = 0.0
    rg = plan.r().cpu().numpy()
    rows = np.array([F * K2 + j for F in faces for j in range(K2)])
    for row in rows:
        a = ref.H.getrow(row).toarray().ravel()
        b = Hg.getrow(row).toarray().ravel()
        eH = max(eH, np.abs(a - b).max() / np.abs(a).max())
        er = max(er, abs(ref.r[row] - rg[row]) / np.abs(ref.r).max())
    nH = sp.linalg.norm(ref.H[rows] - Hg[rows]) / sp.linalg.norm(ref.H[rows])
    nr = np.linalg.norm(ref.r[rows] - rg[rows]) / np.linalg.norm(ref.r[rows])
    u_ref = ohyb.recover(ref, prob.mesh.xyz, prob.mesh.e2v, prob.alpha, prob.beta, prob.f, lam_np, elements=els)
    u = plan.recover(lam_np).cpu().numpy()[els]
    eu = np.abs(u - u_ref).max() / np.abs(u_ref).max()
    nu = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    return {"H_row_rel": eH, "r_rel_to_max": er, "u_rel": eu,
            "normwise": {"H": nH, "r": nr, "u": nu},
            "sample": f"{len(faces)} faces' rows of H and r, {len(els)} elements' u"}


def time_plan(plan, alpha, beta, f, lam, u, steps, warmup):
    """Wall time per setup + recovery step on the plan's stream, and the
    HIP-event times of the setup and recovery kernels."""
    import torch
    for _ in range(warmup):
        plan.setup(alpha, beta, f)
        plan.recover(lam, u)
    torch.cuda.synchronize()
    plan.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.setup(alpha, beta, f)
        plan.recover(lam, u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = plan.timing_read()
    plan.timing(False)
    rc, det = plan.status()
    assert rc == 0, (rc, det)
    return dt / steps, kt["setup_ms"] / max(kt["setup_n"], 1), kt["recover_ms"] / max(kt["recover_n"], 1)


def mixed_leg(args, prob, lam, plain_value):
    """The mixed-precision form on the same workload and lambda: FP32 element
    factor and solves with FP64 refinement (per element until the backward-
    error test passes), and the same with no refinement; throughput and error
    against the oracle for both."""
    import torch

    from paper_1801_08914_amd import Plan
    dev = torch.device("cuda:0")
    alpha, beta, f = (torch.as_tensor(x, device=dev) for x in (prob.alpha, prob.beta, prob.f))
    out = {}
    for name, sweeps in (("refined", None), ("unrefined", 0)):
        plan = Plan(prob.mesh.xyz, prob.mesh.e2v, prob.k, precision="mixed", sweeps=sweeps).bind("cuda:0")
        u = torch.empty((prob.mesh.ne, plan.n), dtype=torch.float64, device=dev)
        plan.setup(alpha, beta, f)
        step_s, setup_ms, rec_ms = time_plan(plan, alpha, beta, f, lam, u, args.steps, args.warmup)
        leg = {"value": prob.mesh.ne / step_s, "unit": "elements/s", "ms_per_step": step_s * 1e3,
               "setup_kernel_ms": setup_ms, "recover_kernel_ms": rec_ms,
               "sweeps": "adaptive (backward-error test, at most 30)" if sweeps is None else sweeps, "vs_fp64_plain": prob.mesh.ne / step_s / plain_value}
        if not args.no_parity:
            leg["error_vs_oracle"] = parity_sample(prob, plan, lam.cpu().numpy())
        out[name] = leg
        del plan, u
        torch.cuda.empty_cache()
    return out


def static_leg(args, prob, plain_value, u_hyb):
    """Static condensation (Sec. 3.1) on the same workload: setup of S and its
    load + recovery throughput, the PCG iterations on S (against those on H)
    and the distance of its u from the hybridized u."""
    import torch

    from paper_1801_08914_amd import Plan
    dev = torch.device("cuda:0")
    alpha, beta, f = (torch.as_tensor(x, device=dev) for x in (prob.alpha, prob.beta, prob.f))
    plan = Plan(prob.mesh.xyz, prob.mesh.e2v, prob.k, system="static").bind("cuda:0")
    plan.setup(alpha, beta, f)
    t0 = time.perf_counter()
    x, info = plan.pcg(1e-12, 20000)
    torch.cuda.synchronize()
    pcg_ms = (time.perf_counter() - t0) * 1e3
    u = torch.empty((prob.mesh.ne, plan.n), dtype=torch.float64, device=dev)
    step_s, setup_ms, rec_ms = time_plan(plan, alpha, beta, f, x, u, args.steps, args.warmup)
    uh = u_hyb.cpu().numpy()
    du = float(np.abs(u.cpu().numpy() - uh).max() / np.abs(uh).max())
    out = {"value": prob.mesh.ne / step_s, "unit": "elements/s", "ms_per_step": step_s * 1e3,
           "setup_kernel_ms": setup_ms, "recover_kernel_ms": rec_ms, "vs_hybridization": prob.mesh.ne / step_s / plain_value,
           "pcg": {"iters": info["iters"], "rel_res": info["rel_res"], "ms": pcg_ms},
           "u_vs_hybridized_rel": du}
    del plan, u
    torch.cuda.empty_cache()
    return out


def _batch_run_timed(b, steps, warmup):
    """Warm-up, then `steps` timed setup + recovery passes of a batch (graph
    replays), with HIP-event times of the two phases."""
    import torch
    for _ in range(warmup):
        b.setup()
        b.recover()
    torch.cuda.synchronize()
    b.timing(True)
    ts = []
    for _ in range(steps):
        t1 = time.perf_counter()
        b.setup()
        b.recover()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    kt = b.timing_read()
    b.timing(False)
    return np.array(ts), kt["setup_ms"] / max(kt["setup_n"], 1), kt["recover_ms"] / max(kt["recover_n"], 1)


def _c4_parity(probs, plans, lams, picks):
    """Worst sampled error of the batch's H rows, r and u against the oracle
    over the picked problems (one of each order)."""
    worst = {"H_row_rel": 0.0, "r_rel_to_max": 0.0, "u_rel": 0.0}
    per = {}
    for i in picks:
        e = parity_sample(probs[i], plans[i], lams[i], nface=16, nel=16)
        per[probs[i].name] = {key: e[key] for key in worst}
        for key in worst:
            worst[key] = max(worst[key], e[key])
    worst["problems"] = per
    return worst


def _copy_calibration():
    """One plain 256 MiB device copy (the reference for the HBM counters)."""
    import torch
    src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def measured_peaks():
    """What the chip reaches on plain work, beside the published peaks: a
    1 GiB device-to-device copy (HBM read + write) and an FP64 8192^3 matrix
    product from the vendor BLAS through torch (matrix cores), each the best
    of five timed repetitions (HIP events on torch's stream)."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best_ms(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            ev0.record()
            fn()
            ev1.record()
            ev1.synchronize()
            ms = ev0.elapsed_time(ev1)
            best = ms if best is None else min(best, ms)
        return best

    n = 128 * 1024 * 1024   # doubles: 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    copy_ms = best_ms(lambda: dst.copy_(src))
    del src, dst
    m = 8192
    a = torch.randn(m, m, dtype=torch.float64, device="cuda:0")
    b = torch.randn(m, m, dtype=torch.float64, device="cuda:0")
    c = torch.empty_like(a)
    gemm_ms = best_ms(lambda: torch.matmul(a, b, out=c), reps=3)
    del a, b, c
    torch.cuda.empty_cache()
    hbm = 2.0 * 8 * n / (copy_ms * 1e-3)
    dgemm = 2.0 * m ** 3 / (gemm_ms * 1e-3)
    return {"hbm_copy_gbs": hbm / 1e9, "hbm_copy_frac_of_peak": hbm / HBM_PEAK,
            "dgemm_tflops": dgemm / 1e12, "dgemm_frac_of_peak": dgemm / FP64_PEAK,
            "how": "1 GiB device copy (read + write bytes); FP64 8192^3 torch.matmul; best of 5 / 3"}


def run_c4(args):
    """The uneven batch (64 jittered problems, n in 8..24, k in 0..3): setup +
    recovery of every problem, a few launches per order and phase (up to
    eight problems each), replayed as hipGraphs; the FP64 plain form is the
    line's value, the mixed-precision form a leg beside it.  Recovery uses a
    seeded random lambda (its cost does not depend on the values)."""
    import synth
    probs = synth.config_c4()
    ne = sum(p.mesh.ne for p in probs)
    by_k = {k: sum(p.mesh.ne for p in probs if p.k == k) for k in range(4)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_mix(probs, label="the uneven 64-problem batch")
        print(f"cpu baseline: {cpu['value']:.0f} el/s (1 process), "
              f"{cpu['multi_process']['value']:.0f} el/s ({cpu['multi_process']['cores']} processes)",
              file=sys.stderr, flush=True)

    import torch

    from paper_1801_08914_amd import Batch, Plan
    t0 = time.perf_counter()
    plans = [Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True).bind("cuda:0") for p in probs]
    plan_s = time.perf_counter() - t0
    b = Batch(plans)
    rng = np.random.default_rng(0)
    lams = [rng.standard_normal(max(pl.m, 1)) for pl in plans]
    for i, p in enumerate(probs):
        b.set(i, p.alpha, p.beta, p.f, lam=lams[i])
    if args.tiles:
        tiles = tuple(int(x) for x in args.tiles.split(","))
        b.tiles(*tiles)
    else:
        tiles = b.autotune(reps=1)
    b.graph(True)
    ts, setup_ms, rec_ms = _batch_run_timed(b, args.steps, args.warmup)
    if args.copy_calib:
        _copy_calibration()
    for i, pl in enumerate(plans):
        rc, det = pl.status()
        assert rc == 0, (i, rc, det)
    value = ne * len(ts) / ts.sum()
    print(f"c4 fp64: {value:.0f} el/s, setup phase {setup_ms:.2f} ms, recovery phase {rec_ms:.2f} ms",
          file=sys.stderr, flush=True)
    flops = sum(algo_counts(p.k)["setup_flops"] * p.mesh.ne for p in probs)
    rbytes = sum(algo_counts(p.k)["recover_bytes"] * p.mesh.ne for p in probs)
    roof = {"bound": "mfma", "kernel": "setup phase: k_batch_zero, then k_setup_multi<3>, <2>, <1>, <0> (up to "
                                        "eight problems per launch)",
            "achieved": flops / (setup_ms * 1e-3) / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": flops / (setup_ms * 1e-3) / FP64_PEAK,
            "traffic": traffic_from_profile("setup", ne, "hbm_traffic_uneven_batch_64.json"),
            "phase_ms": setup_ms, "algorithmic_flops": flops,
            "flops_per_element_by_order": {k: algo_counts(k)["setup_flops"] for k in range(4)},
            "recover_phase_ms": rec_ms, "recover_hbm_gbs": rbytes / (rec_ms * 1e-3) / 1e9,
            "recover_hbm_frac": rbytes / (rec_ms * 1e-3) / HBM_PEAK,
            "recover_traffic": traffic_from_profile("recover", ne, "hbm_traffic_uneven_batch_64.json")}
    picks = [next(i for i, p in enumerate(probs) if p.k == k) for k in range(4) if any(p.k == k for p in probs)]
    parity = None if args.no_parity else _c4_parity(probs, plans, lams, picks)
    del b, plans
    torch.cuda.empty_cache()
    mixed = None if args.no_mixed else c4_mixed_leg(args, probs, tiles, ne, value, lams, picks)
    out = {"metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * ts.mean(), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "uneven batch: 64 jittered n^3 problems, n~U{8..24}, k~U{0..3}, alpha and beta "
                                  "lognormal per problem, seed 4",
                      "elements": ne, "elements_by_order": by_k, "problems": len(probs),
                      "precision": "fp64-plain",
                      "launch": "per order and phase, launches of up to eight problems (descriptors in the "
                                "kernel arguments), hipGraph replay"},
           "step_ms_p50": 1e3 * float(np.median(ts)), "step_ms_p90": 1e3 * float(np.percentile(ts, 90)),
           "host_planning_s": plan_s, "roofline": roof}
    if parity is not None:
        out["error_vs_oracle"] = parity
    out["mixed"] = mixed
    if not (args.no_peaks or args.copy_calib):   # (counter runs: the calibration copy stays the largest)
        pk = measured_peaks()
        roof["measured_peaks"] = pk
        roof["frac_of_measured_dgemm"] = roof["achieved"] / pk["dgemm_tflops"]
        roof["recover_frac_of_measured_copy"] = rbytes / (rec_ms * 1e-3) / (pk["hbm_copy_gbs"] * 1e9)
        print(f"measured peaks: copy {pk['hbm_copy_gbs']:.0f} GB/s, FP64 GEMM {pk['dgemm_tflops']:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
    if cpu is not None:
        cpu["gpu_over_cpu"] = value / cpu["value"]
        out["cpu_baseline"] = cpu
    return out


def c4_mixed_leg(args, probs, tiles, ne, plain_value, lams, picks):
    """The same uneven batch with every problem in the mixed-precision form
    (FP32 element factors and solves, FP64 refinement), refined (adaptive
    sweeps with the backward-error test) and unrefined: one persistent
    launch per phase over the mixed problems' items, hipGraph replay, tiles
    from the library's autotuner on the unrefined batch (or --tiles).
    Problems with an element that needed the FP64 fallback are counted (the
    result is still within the bound), failures too."""
    import torch

    from paper_1801_08914_amd import Batch, Plan
    out = {}
    tiles = tuple(int(x) for x in args.tiles.split(",")) if args.tiles else None
    for name, sweeps in (("unrefined", 0), ("refined", None)):
        plans = [Plan(p.mesh.xyz, p.mesh.e2v, p.k, generic=True, precision="mixed", sweeps=sweeps).bind("cuda:0")
                 for p in probs]
        b = Batch(plans)
        for i, p in enumerate(probs):
            b.set(i, p.alpha, p.beta, p.f, lam=lams[i])
        if tiles is None:
            tiles = b.autotune(reps=1)
        b.tiles(*tiles)
        b.graph(True)
        steps = max(1, min(args.steps, 5))
        ts, setup_ms, rec_ms = _batch_run_timed(b, steps, 1)
        failed = [i for i, pl in enumerate(plans) if pl.status()[0] != 0]
        val = ne * len(ts) / ts.sum()
        leg = {"value": val, "unit": "elements/s", "ms_per_step": 1e3 * ts.mean(), "steps": len(ts),
               "vs_fp64_plain": val / plain_value, "setup_phase_ms": setup_ms, "recover_phase_ms": rec_ms,
               "sweeps": "adaptive (backward-error test, at most 30)" if sweeps is None else sweeps,
               "problems_failed": len(failed), "tiles": {"blocks_per_cu": tiles[0], "items_per_block": tiles[1]}}
        if hasattr(plans[0], "fallback_count"):
            leg["elements_fp64_fallback"] = int(sum(pl.fallback_count() for pl in plans))
        if not args.no_parity and not failed:
            leg["error_vs_oracle"] = _c4_parity(probs, plans, lams, picks)
        print(f"c4 mixed {name}: {val:.0f} el/s, setup phase {setup_ms:.1f} ms, failed problems {len(failed)}",
              file=sys.stderr, flush=True)
        out[name] = leg
        del b, plans
        torch.cuda.empty_cache()
    return out


def run_single(args, prob, label):
    """Setup + recovery of one problem through the plan (C1: latency of the
    tiny RT0 problem; C3: the RT2 48^3 jittered workload on the generic
    kernels), timed over the steps; lambda from one PCG solve."""
    import torch

    from paper_1801_08914_amd import Plan
    ne = prob.mesh.ne
    plan = Plan(prob.mesh.xyz, prob.mesh.e2v, prob.k).bind("cuda:0")
    dev = torch.device("cuda:0")
    alpha, beta, f = (torch.as_tensor(x, device=dev) for x in (prob.alpha, prob.beta, prob.f))
    u = torch.empty((ne, plan.n), dtype=torch.float64, device=dev)
    plan.setup(alpha, beta, f)
    lam, info = plan.pcg(1e-12, 20000)
    for _ in range(args.warmup):
        plan.setup(alpha, beta, f)
        plan.recover(lam, u)
    torch.cuda.synchronize()
    plan.timing(True)
    ts = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        plan.setup(alpha, beta, f)
        plan.recover(lam, u)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    kt = plan.timing_read()
    rc, det = plan.status()
    assert rc == 0, (rc, det)
    ts = np.array(ts)
    parity = None if args.no_parity else parity_sample(prob, plan, lam.cpu().numpy())
    m_, nnz_ = plan.m, plan.nnz
    value = ne * len(ts) / ts.sum()
    stat = None if args.no_static else static_leg(args, prob, value, plan.recover(lam))
    del plan, u
    mixed = None if args.no_mixed else mixed_leg(args, prob, lam, value)
    out = {"metric": METRIC, "value": ne * len(ts) / ts.sum(), "unit": "elements/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * ts.mean(), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": label, "elements": ne, "k": prob.k, "m": m_, "nnz": nnz_,
                      "precision": "fp64-plain"},
           "step_us_p50": 1e6 * float(np.median(ts)), "step_us_p90": 1e6 * float(np.percentile(ts, 90)),
           "setup_kernel_ms": kt["setup_ms"] / max(kt["setup_n"], 1),
           "recover_kernel_ms": kt["recover_ms"] / max(kt["recover_n"], 1),
           "pcg": {"iters": info["iters"], "rel_res": info["rel_res"]}}
    if parity is not None:
        out["error_vs_oracle"] = parity
    if mixed is not None:
        out["mixed"] = mixed
    if stat is not None:
        out["static_condensation"] = stat
    t_set = out["setup_kernel_ms"] * 1e-3
    if t_set > 0:
        fl = algo_counts(prob.k)["setup_flops"] * ne
        out["roofline"] = {"bound": "mfma", "kernel": f"k_setup_generic<{prob.k}> (+ zeroing of the same-face blocks)",
                           "achieved": fl / t_set / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                           "frac": fl / t_set / FP64_PEAK, "traffic": None}
    return out


def solve_phases(prob, steps=3):
    """Setup (matrix and load), Jacobi-PCG (rtol 1e-12) and recovery of one
    problem: HIP-event kernel times of setup and recovery (mean over steps),
    PCG wall time and iterations, and the time to solution (the paper's
    tables: formation of the reduced system + solve + back substitution)."""
    import torch

    from paper_1801_08914_amd import Plan
    dev = torch.device("cuda:0")
    alpha, beta, f = (torch.as_tensor(x, device=dev) for x in (prob.alpha, prob.beta, prob.f))
    plan = Plan(prob.mesh.xyz, prob.mesh.e2v, prob.k).bind("cuda:0")
    plan.setup(alpha, beta, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, info = plan.pcg(1e-12, 200000)
    torch.cuda.synchronize()
    pcg_s = time.perf_counter() - t0
    u = torch.empty((prob.mesh.ne, plan.n), dtype=torch.float64, device=dev)
    step_s, setup_ms, rec_ms = time_plan(plan, alpha, beta, f, lam, u, steps, 1)
    out = {"elements": prob.mesh.ne, "k": prob.k, "m": plan.m, "setup_ms": setup_ms, "recover_ms": rec_ms,
           "pcg_ms": pcg_s * 1e3, "pcg_iters": info["iters"], "converged": info["converged"],
           "time_to_solution_ms": setup_ms + pcg_s * 1e3 + rec_ms,
           "elements_per_s": prob.mesh.ne / ((setup_ms + rec_ms) * 1e-3)}
    del plan, u
    torch.cuda.empty_cache()
    return out


def run_softhard(args):
    """The soft-hard materials study of Sec. 6.1 on one GPU: RT0 64x64x32,
    RT1 32x32x16 and RT3 16x16x8 (the paper's initial meshes), alpha = 10^p
    in the inclusions for p in {-8, -4, 0, 4, 8}; Jacobi-PCG (the paper's AMG
    is out of scope, so iteration counts are not comparable)."""
    import synth
    rows = []
    for k in (0, 1, 3):
        for p in synth.SOFTHARD_EXPONENTS:
            r = solve_phases(synth.config_softhard(k, p), steps=args.steps)
            r["p"] = p
            rows.append(r)
            print(json.dumps({"progress": f"RT{k} p={p}", **{x: r[x] for x in ("pcg_iters", "time_to_solution_ms")}}),
                  file=sys.stderr, flush=True)
    el = sum(r["elements"] for r in rows)
    t = sum((r["setup_ms"] + r["recover_ms"]) * 1e-3 for r in rows)
    out = {"metric": METRIC, "value": el / t, "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": 1e3 * t / len(rows), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "soft-hard materials: RT0 64x64x32, RT1 32x32x16, RT3 16x16x8, alpha = 10^p "
                                  "in [1/4,1/2]^3 u [1/2,3/4]^3, p in {-8,-4,0,4,8}, beta = 1, f = (1,1,1)",
                      "precision": "fp64-plain", "preconditioner": "Jacobi"},
           "runs": rows}
    print(json.dumps(out), flush=True)


def run_spe10(args):
    """The SPE10-shaped stand-in of Sec. 6.4 (RT0, 60x220x85 cells of
    20x10x2, layered heavy-tailed coefficient): the per-phase times of the
    paper's table (hybridize, PCG solve, back substitution, total)."""
    import synth
    prob = synth.config_spe10_standin()
    r = solve_phases(prob, steps=args.steps)
    out = {"metric": METRIC, "value": r["elements_per_s"], "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": r["setup_ms"] + r["recover_ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "SPE10-shaped stand-in: RT0 60x220x85, cells 20x10x2, layered lognormal alpha "
                                  "(sigma 1 / 2), beta = 1, seed 10", "precision": "fp64-plain",
                      "preconditioner": "Jacobi"},
           "phases_ms": {"hybridize": r["setup_ms"], "pcg_solve": r["pcg_ms"], "back_substitution": r["recover_ms"],
                         "total": r["time_to_solution_ms"]},
           "pcg": {"iters": r["pcg_iters"], "converged": r["converged"]}, "m": r["m"]}
    print(json.dumps(out), flush=True)


def run_c5(args):
    """The serving stream: Poisson arrivals of hybridization requests (jittered
    meshes, k in 1..3, 1..8 right-hand sides reusing the factors).  First the
    saturation throughput (every request queued at once), then the stream at
    0.7 of it in real time; p50/p99 latency = completion - arrival."""
    import synth
    from paper_1801_08914_amd.serving import Request, Server, latency_stats, run_stream

    def stream(qps):
        return [(t, Request(p.mesh.xyz, p.mesh.e2v, p.k, p.alpha, p.beta, fs, tag=p.name))
                for t, p, fs in synth.serving_requests(args.requests, qps, nmin=args.nmin, nmax=args.nmax)]

    budget = int(args.budget_gb * 2**30)
    srv = Server(budget, slots=args.slots, rtol=1e-12)
    sat = latency_stats(run_stream(srv, stream(1.0), realtime=False))
    srv.close()
    qps = 0.7 * sat["req_per_s"]
    srv = Server(budget, slots=args.slots, rtol=1e-12)
    res = run_stream(srv, stream(qps), realtime=True)
    srv.close()
    st = latency_stats(res)
    out = {"metric": METRIC, "value": st["element_solves_per_s"], "unit": "element-solves/s", "n_gpus": 1,
           "steps": len(res), "warmup": 0, "ms_per_step": 1e3 * st["mean_s"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"serving stream: {args.requests} requests, jittered n^3 meshes "
                                  f"n~U{{{args.nmin}..{args.nmax}}}, k~U{{1..3}}, 1..8 rhs per request, seed 5",
                      "slots": args.slots, "budget_gb": args.budget_gb, "qps": qps,
                      "saturation_req_per_s": sat["req_per_s"], "precision": "fp64-plain"},
           "latency_p50_s": st["p50_s"], "latency_p99_s": st["p99_s"], "req_per_s": st["req_per_s"],
           "saturation": sat}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-static", action="store_true", help="skip the static-condensation leg")
    ap.add_argument("--skip-solve", action="store_true",
                    help="recover from a seeded random lambda instead of the PCG solution (profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--config", default="c4", choices=["c1", "c2", "c3", "c4", "c5", "softhard", "spe10"],
                    help="c4: the uneven 64-problem batch (default line, with C2 and C3 legs); c1: RT0 4^3 "
                         "latency; c2: RT1 32^3; c3: RT2 48^3 jittered; c5: the serving stream; softhard: the "
                         "soft-hard materials study; spe10: the SPE10-shaped stand-in")
    ap.add_argument("--no-legs", action="store_true", help="c4: skip the C2 and C3 legs")
    ap.add_argument("--no-peaks", action="store_true", help="c4: skip the measured copy / FP64 GEMM peaks")
    ap.add_argument("--tiles", default="", help="c4: fixed batch tiles 'blocks_per_cu,items_per_block' "
                                                "instead of the autotuner's (profiling runs)")
    ap.add_argument("--requests", type=int, default=40, help="c5: requests in the stream")
    ap.add_argument("--nmin", type=int, default=8, help="c5: smallest mesh edge")
    ap.add_argument("--nmax", type=int, default=16, help="c5: largest mesh edge")
    ap.add_argument("--slots", type=int, default=4, help="c5: requests in flight")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="c5: device-memory budget")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the sharding of the path across GPUs is a design only)"}))
        sys.exit(2)

    if args.config == "c4":
        out = run_c4(args)
        if not args.no_legs:
            import copy

            import synth
            leg_args = copy.copy(args)
            leg_args.steps, leg_args.warmup, leg_args.no_static = min(args.steps, 10), 2, True
            leg_args.no_cpu_baseline = True
            legs = {}
            for name, fn in (("c2", lambda: run_c2(leg_args)),
                             ("c3", lambda: run_single(leg_args, synth.config_c3(), C3_LABEL))):
                t0 = time.perf_counter()
                r = fn()
                for key in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data", "unit"):
                    r.pop(key, None)
                r["wall_s"] = time.perf_counter() - t0
                legs[name] = r
                print(f"leg {name}: {r['value']:.0f} el/s", file=sys.stderr, flush=True)
            out["legs"] = legs
        print(json.dumps(out), flush=True)
        return
    if args.config == "softhard":
        run_softhard(args)
        return
    if args.config == "spe10":
        run_spe10(args)
        return
    if args.config == "c5":
        run_c5(args)
        return
    if args.config in ("c1", "c3"):
        import synth
        if args.config == "c1":
            out = run_single(args, synth.config_c1(), "rt0_4x4x4 RT0 unit cube 4^3, alpha = beta = 1, seed 1")
        else:
            out = run_single(args, synth.config_c3(), C3_LABEL)
        print(json.dumps(out), flush=True)
        return
    print(json.dumps(run_c2(args)), flush=True)


C3_LABEL = "rt2_48x48x48 RT2 jittered 0.2h, alpha lognormal clipped [1e-2,1e2], beta = 1e-2, seed 3"


def run_c2(args):
    """RT1 on the structured 32^3 mesh (affine: the RT1-specific kernels)."""
    import torch

    import synth
    from paper_1801_08914_amd import Plan

    prob = synth.config_c2()
    k, ne = prob.k, prob.mesh.ne
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_mix([prob], label="the RT1 32^3 workload")
    plan = Plan(prob.mesh.xyz, prob.mesh.e2v, k).bind("cuda:0")
    dev = torch.device("cuda:0")
    alpha = torch.as_tensor(prob.alpha, device=dev)
    beta = torch.as_tensor(prob.beta, device=dev)
    f = torch.as_tensor(prob.f, device=dev)
    u = torch.empty((ne, plan.n), dtype=torch.float64, device=dev)

    # lambda for the recovery: one Jacobi-PCG solve (not part of the metric)
    plan.setup(alpha, beta, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.skip_solve:
        lam = torch.as_tensor(np.random.default_rng(0).standard_normal(plan.m), device=dev)
        info = {"iters": 0, "rel_res": None}
    else:
        lam, info = plan.pcg(1e-12, 20000)
    torch.cuda.synchronize()
    pcg_ms = (time.perf_counter() - t0) * 1e3
    if args.copy_calib:
        _copy_calibration()
    rc, det = plan.status()
    assert rc == 0, (rc, det)

    for _ in range(args.warmup):
        plan.setup(alpha, beta, f)
        plan.recover(lam, u)
    torch.cuda.synchronize()
    plan.timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.setup(alpha, beta, f)
        plan.recover(lam, u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = plan.timing_read()
    plan.timing(False)
    rc, det = plan.status()
    assert rc == 0, (rc, det)

    ms_step = dt * 1e3 / args.steps
    value = ne * args.steps / dt
    cnt = per_element_counts(k, ne, plan.nnz, plan.m, prob.mesh.nv)
    t_setup = kt["setup_ms"] / max(kt["setup_n"], 1) * 1e-3
    t_rec = kt["recover_ms"] / max(kt["recover_n"], 1) * 1e-3
    B = cnt["setup_bytes"] * ne
    Fl = cnt["setup_flops"] * ne
    hbm_frac = B / t_setup / HBM_PEAK
    fp_frac = Fl / t_setup / FP64_PEAK
    bound = "hbm" if B / HBM_PEAK >= Fl / FP64_PEAK else "alu"
    roof = {"bound": bound, "kernel": "k_setup_k1 + k_finalize_k1 (assembly, condensation, H_T/r scatter)",
            "achieved": B / t_setup / 1e9 if bound == "hbm" else Fl / t_setup / 1e12,
            "peak": 8000.0 if bound == "hbm" else 78.6,
            "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
            "frac": hbm_frac if bound == "hbm" else fp_frac,
            "traffic": _sum_or_none(traffic_from_profile("k_setup_k1", ne), traffic_from_profile("k_finalize_k1", ne)),
            "kernel_ms": t_setup * 1e3,
            "fp64_achieved_tflops": Fl / t_setup / 1e12, "fp64_frac": fp_frac,
            "hbm_achieved_gbs": B / t_setup / 1e9, "hbm_frac": hbm_frac,
            "recover_kernel_ms": t_rec * 1e3,
            "recover_hbm_gbs": cnt["recover_bytes"] * ne / t_rec / 1e9,
            "recover_traffic": traffic_from_profile("k_recover_k1", ne),
            "bytes_per_element": cnt["setup_bytes"], "flops_per_element": cnt["setup_flops"]}
    out = {"metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": prob.name + " RT1 structured 32^3, alpha lognormal(0,1), beta=1, f~N(0,1), seed 2",
                      "elements": ne, "k": k, "m": plan.m, "nnz": plan.nnz, "precision": "fp64-plain"},
           "pcg": {"iters": info["iters"], "rel_res": info["rel_res"], "ms": pcg_ms},
           "roofline": roof}
    if not args.no_parity:
        out["error_vs_oracle"] = parity_sample(prob, plan, lam.cpu().numpy())
    del plan
    torch.cuda.empty_cache()
    if not args.no_mixed:
        out["mixed"] = mixed_leg(args, prob, lam, value)
    if not args.no_static:
        out["static_condensation"] = static_leg(args, prob, value, u)
    if cpu is not None:
        cpu["gpu_over_cpu"] = value / cpu["value"]
        out["cpu_baseline"] = cpu
    return out


if __name__ == "__main__":
    main()
