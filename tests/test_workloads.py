"""Synthetic workload generators: shapes, seeding, sizes."""
import numpy as np

import workloads as wl


def test_path_22x20_shapes_and_seed():
    s1, f1 = wl.path_22x20(50)
    s2, f2 = wl.path_22x20(50)
    assert s1.landmarks.shape == (20, 22, 3) and s1.landmarks.dtype == np.float64
    assert f1.shape == (50, 22, 3)
    assert np.array_equal(s1.landmarks, s2.landmarks) and np.array_equal(f1, f2)
    assert np.array_equal(f1[0], s1.waypoints[0])


def test_path_300x500_shapes():
    s, f = wl.path_300x500(100)
    assert s.landmarks.shape == (500, 300, 3) and s.landmarks.dtype == np.float32
    assert f.shape == (100, 300, 3) and f.dtype == np.float32
    step = np.diff(f.astype(np.float64), axis=0)
    assert 0.004 < step.std() < 0.006


def test_rigid_small_copy_and_bytes():
    s, base = wl.rigid_5000x10000(n_atoms=64, n_landmarks=10)
    assert s.landmarks.shape == (10, 64, 3)
    fr = wl.rigid_frames(base, 3)
    assert fr.shape == (3, 64, 3)
    # Full size: 10,000 landmarks x 5,000 atoms x 12 B = 600 MB of FP32.
    assert 10_000 * 5_000 * 12 == 600_000_000


def test_walkers_ranges():
    ws = wl.walkers(n_walkers=6, n_frames=2)
    assert len(ws) == 6
    for w in ws:
        assert 50 <= w.system.n_atoms <= 2000
        assert 200 <= w.system.n_landmarks <= 5000
        assert w.frames.shape == (2, w.system.n_atoms, 3)
    ws2 = wl.walkers(n_walkers=6, n_frames=2)
    assert all(np.array_equal(a.system.landmarks, b.system.landmarks) for a, b in zip(ws, ws2))


def test_rigid_copy():
    x = np.random.default_rng(0).normal(size=(5, 3))
    y, R, t = wl.rigid_copy(x, 3)
    assert np.allclose(R @ R.T, np.eye(3)) and abs(np.linalg.det(R) - 1) < 1e-12
    assert np.allclose(y, x @ R.T + t)
