"""The seeded generators are deterministic and produce the documented geometry."""
import numpy as np

from paper_1707_09898_amd import workloads as wl


def test_seeded_and_deterministic():
    a, b = wl.config2(), wl.config2()
    assert np.array_equal(a.rho, b.rho)
    assert a.rho.shape == (64, 64, 64)
    assert 0.0 <= a.rho.min() and a.rho.max() <= 1.0


def test_box_filter_preserves_constants_and_is_count_normalized():
    u = np.full((5, 6, 7), 0.3)
    assert np.allclose(wl.box_filter3(u), 0.3)
    v = np.zeros((3, 3, 3))
    v[0, 0, 0] = 8.0
    assert abs(wl.box_filter3(v)[0, 0, 0] - 1.0) < 1e-15   # 8 in-grid neighbours


def test_config_geometry():
    c1 = wl.config1()
    assert c1.n == (16, 16, 18) and c1.sensor == (8, 9, 4, 12, 17, 18)
    c3 = wl.config3()
    assert c3.rho.shape == (128, 256, 256) and c3.design[5] == 124 and c3.sensor[4] == 127
    c4 = wl.config4()
    assert np.allclose(np.linalg.norm(c4.m0_field, axis=0), 1.0)
    assert c4.h_target.shape == (3, 4, 32, 32) and np.abs(c4.h_target).max() <= 0.05 + 1e-15
    batch = wl.config5()
    assert len(batch) == 64
    for w in batch:
        nx, ny, nz = w.n
        assert 32 <= nx <= 160 and 32 <= ny <= 160 and 32 <= nz <= 96
        assert w.p in (3, 4) and all(0.5 <= v <= 2.0 for v in w.h)
        assert w.sensor[4] == nz // 2 + 3
