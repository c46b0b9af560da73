"""Host-side checks of the boundary options (no GPU): quad_q, natural
boundary faces (hyb_mesh.ess) and hyb_get_csr before binding."""
import ctypes
import os

import numpy as np
import pytest

import synth
from oracle import topology as otopo


def _lib():
    from paper_1801_08914_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libhyb.so not built")
    return _abi.load_library()


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_quad_q_only_the_built_rule(k):
    _lib()
    from paper_1801_08914_amd import HybError, Plan, _abi
    mesh = synth.structured_hex(2)
    for q in (0, k + 2):
        Plan(mesh.xyz, mesh.e2v, k, quad_q=q)
    for q in (k + 1, k + 3, -1):
        with pytest.raises(HybError) as ei:
            Plan(mesh.xyz, mesh.e2v, k, quad_q=q)
        assert ei.value.code == _abi.HYB_E_ARG


def test_natural_faces_keep_the_topology():
    """Natural faces carry no multiplier, like essential ones: faces, frames,
    multipliers and the CSR pattern of H do not depend on the mask."""
    _lib()
    from paper_1801_08914_amd import Plan
    rng = np.random.default_rng(4)
    mesh, _ = synth.rotate_connectivity(synth.structured_hex(3, jitter=0.2, rng=rng), rng)
    ess = rng.integers(0, 2, size=(mesh.ne, 6)).astype(np.uint8)
    t0 = Plan(mesh.xyz, mesh.e2v, 2).topology()
    t1 = Plan(mesh.xyz, mesh.e2v, 2, ess=ess).topology()
    for key in t0:
        assert np.array_equal(t0[key], t1[key]), key
    ref = otopo.build_topology(mesh.e2v)
    assert np.array_equal(t1["elem_face"], ref.elem_face)


def test_natural_faces_rejected_by_static_condensation():
    _lib()
    from paper_1801_08914_amd import HybError, Plan, _abi
    mesh = synth.structured_hex(2)
    ess = np.ones((mesh.ne, 6), np.uint8)
    Plan(mesh.xyz, mesh.e2v, 1, system="static", ess=ess)          # all essential: fine
    ess[0, 0] = 0                                                   # face 0 of element 0 is on the boundary
    with pytest.raises(HybError) as ei:
        Plan(mesh.xyz, mesh.e2v, 1, system="static", ess=ess)
    assert ei.value.code == _abi.HYB_E_ARG
    with pytest.raises(ValueError):
        Plan(mesh.xyz, mesh.e2v, 1, ess=np.ones((mesh.ne - 1, 6), np.uint8))


def test_get_csr_needs_bound_buffers():
    lib = _lib()
    from paper_1801_08914_amd import HybError, Plan, _abi
    mesh = synth.structured_hex(2)
    p = Plan(mesh.xyz, mesh.e2v, 1)
    with pytest.raises(HybError) as ei:
        p.csr_pointers()
    assert ei.value.code == _abi.HYB_E_STATE
    assert lib.hyb_get_csr(None, None, None, None, None, None) == _abi.HYB_E_ARG
    assert lib.hyb_solve(None, None, None, ctypes.c_double(1e-12), 10, None, None, None) == _abi.HYB_E_ARG
    assert lib.hyb_pcg(None, ctypes.c_double(1e-12), 10, None, None) == _abi.HYB_E_ARG
