"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def row_rel_err(H_ref, val_gpu):
    """max over rows of ||dH_row||_inf / ||H_row||_inf (same CSR pattern)."""
    d = np.abs(H_ref.data - val_gpu)
    worst = 0.0
    for i in range(H_ref.shape[0]):
        a, b = H_ref.indptr[i], H_ref.indptr[i + 1]
        if b > a:
            worst = max(worst, d[a:b].max() / max(np.abs(H_ref.data[a:b]).max(), 1e-300))
    return worst


def rel_inf(ref, got):
    ref = np.asarray(ref)
    got = np.asarray(got)
    if ref.size == 0:
        return 0.0
    return float(np.abs(ref - got).max() / max(np.abs(ref).max(), 1e-300))


def gpu_setup(prob_mesh, k, alpha, beta, f=None, g=None):
    torch = require_gpu()
    from paper_1801_08914_amd import Plan
    plan = Plan(prob_mesh.xyz, prob_mesh.e2v, k).bind()
    plan.setup(alpha, beta, f, g)
    torch.cuda.synchronize()
    rc, det = plan.status()
    assert rc == 0, (rc, det)
    return plan


def norm_rel(ref, got):
    """||ref - got||_2 / ||ref||_2 (Frobenius for matrices / CSR value arrays)."""
    ref = np.asarray(ref, dtype=np.float64).ravel()
    got = np.asarray(got, dtype=np.float64).ravel()
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(ref - got) / nr) if nr > 0 else float(np.linalg.norm(got))


def ld_row_errors(Hld: dict, rld: dict, rows, H_a, r_a):
    """Row-relative errors of a FP64 H (scipy CSR) and r against the
    long-double reference dicts, over the given rows."""
    import collections
    byrow = collections.defaultdict(dict)
    for (mu, nu), v in Hld.items():
        byrow[mu][nu] = v
    eH = 0.0
    rmax = max(abs(float(v)) for v in rld.values()) if rld else 1.0
    er = 0.0
    for mu in rows:
        ref = byrow[mu]
        cols = np.array(sorted(ref))
        vref = np.array([float(ref[c]) for c in cols])
        a, b = H_a.indptr[mu], H_a.indptr[mu + 1]
        got = dict(zip(H_a.indices[a:b].tolist(), H_a.data[a:b].tolist()))
        vgot = np.array([got.get(int(c), np.nan) for c in cols])
        eH = max(eH, np.abs(vref - vgot).max() / np.abs(vref).max())
        er = max(er, abs(float(rld[mu]) - r_a[mu]) / rmax)
    return eH, er


def ld_dense(Hld: dict, rld: dict, m: int):
    """Dense float64 copies of the long-double H and r dicts (small m only)."""
    H = np.zeros((m, m))
    for (mu, nu), v in Hld.items():
        H[mu, nu] = float(v)
    r = np.zeros(m)
    for mu, v in rld.items():
        r[mu] = float(v)
    return H, r


U64 = 2.0 ** -53


def kappa_of(k, mesh, alpha, beta, topo, elements=None, ess=None):
    """kappa_s = max cond_2 of the equilibrated kept element blocks over the
    given elements (all by default), from the oracle (``extended.kappa_scaled``)."""
    from oracle import extended as oext
    els = np.arange(mesh.ne) if elements is None else np.asarray(elements)
    return oext.kappa_scaled(k, mesh.xyz, mesh.e2v, alpha, beta, topo, els, ess)


def accuracy_bound(e_oracle: float, kappa: float) -> float:
    """The GPU must be at least as accurate as the FP64 oracle (factor 2 for
    rounding-order luck) against the long-double reference, or within the
    FP64 floor kappa_s 2^-53 of a backward-stable method where the oracle
    happens to be luckier, and never needs to beat 1e-12.  The oracle's own
    error is capped first: more than 10 kappa_s 2^-53 from the long-double
    reference means that one of the two references is wrong, and the bound
    is refused rather than loosened."""
    cap = 10.0 * kappa * U64
    assert e_oracle <= cap, f"FP64 oracle {e_oracle:.2e} off the long-double reference, above 10 kappa_s u = {cap:.2e}"
    return max(1e-12, 2.0 * e_oracle, kappa * U64)


def oracle_gap_bound(kappa: float) -> float:
    """Largest admissible distance between the GPU and the FP64 oracle
    directly: both within 10 kappa_s 2^-53 of the exact values."""
    return 20.0 * kappa * U64


def mixed_bound(e_oracle: float, kappa: float) -> float:
    """The mixed-precision form refined: within max(1e-10, 2 x the FP64
    oracle's own error, the FP64 floor kappa_s 2^-53) of the long-double
    reference (the oracle's error capped as in ``accuracy_bound``)."""
    cap = 10.0 * kappa * U64
    assert e_oracle <= cap, f"FP64 oracle {e_oracle:.2e} off the long-double reference, above 10 kappa_s u = {cap:.2e}"
    return max(1e-10, 2.0 * e_oracle, kappa * U64)
