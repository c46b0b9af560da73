"""Host-side checks of the workload generators (no GPU)."""
import numpy as np

import synth


def test_workload_generators():
    """Shapes and coefficient classes of the generators (host only)."""
    p = synth.config_softhard(1, 4, (8, 8, 4))
    assert p.mesh.ne == 256 and set(np.unique(p.alpha)) == {1.0, 1e4}
    assert np.allclose(p.mesh.xyz.max(axis=0), 1.0)
    s = synth.config_spe10_standin((6, 22, 9))
    assert s.mesh.ne == 6 * 22 * 9 and np.allclose(s.mesh.xyz.max(axis=0), [120.0, 220.0, 18.0])
    assert s.alpha.max() / s.alpha.min() > 1e4
