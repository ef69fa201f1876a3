"""Pins for the FP64 oracle's path variables (Eq. 2 with q_i = i, and z)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.path import landmark_lambda, path_cv, path_sz
from oracle.msd import msd


@pytest.mark.parametrize("seed", range(6))
def test_bounds(seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(2, 400))
    D = rng.uniform(0, 2, L)
    lam = float(rng.uniform(1, 1000))
    r = path_sz(D, lam)
    assert 1.0 <= r.s <= L
    assert D.min() - math.log(L) / lam - 1e-12 <= r.z <= D.min() + 1e-15
    assert abs(r.c.sum()) < 1e-9 * max(1.0, np.abs(r.c).max())
    assert abs(r.p.sum() - 1.0) < 1e-14


def test_all_equal_distances():
    for L in (1, 2, 7, 500):
        D = np.full(L, 0.37)
        r = path_sz(D, 123.0)
        assert r.s == (L + 1) / 2
        assert abs(r.z - (0.37 - math.log(L) / 123.0)) < 1e-15


def test_two_landmarks_closed_form():
    D1, D2, lam = 0.011, 0.019, 250.0
    r = path_sz(np.array([D1, D2]), lam)
    assert abs(r.s - (1 + 1 / (1 + math.exp(lam * (D2 - D1))))) < 1e-15
    assert abs(r.z - (-math.log(math.exp(-lam * D1) + math.exp(-lam * D2)) / lam)) < 1e-15


def test_shift_invariance():
    rng = np.random.default_rng(5)
    D = rng.uniform(0, 0.1, 50)
    a, b = path_sz(D, 300.0), path_sz(D + 0.7, 300.0)
    assert abs(a.s - b.s) < 1e-12
    assert abs((b.z - a.z) - 0.7) < 1e-12


def test_sharp_limit():
    D = np.array([0.3, 0.1, 0.2, 0.25])
    r = path_sz(D, 1e6)
    assert abs(r.s - 2.0) < 1e-12
    assert abs(r.z - 0.1) < 1e-12


def test_arbitrary_property():
    rng = np.random.default_rng(8)
    D = rng.uniform(0, 0.05, 30)
    q = rng.normal(size=30)
    r = path_sz(D, 200.0, q)
    e = [math.exp(-200.0 * d) for d in D]
    assert abs(r.s - math.fsum(qi * ei for qi, ei in zip(q, e)) / math.fsum(e)) < 1e-13


def _fd(fun, x, h=1e-6):
    g = np.zeros_like(x)
    for k in range(x.shape[0]):
        for c in range(3):
            xp = x.copy(); xp[k, c] += h
            xm = x.copy(); xm[k, c] -= h
            g[k, c] = (fun(xp) - fun(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("weights", ["uniform", "equal", "distinct"])
def test_path_gradients_match_finite_differences(weights):
    sysm = wl.small_path(8, 12, seed=3)
    A = sysm.landmarks
    rng = np.random.default_rng(4)
    x = sysm.waypoints[0] + rng.normal(0, 0.02, (8, 3))
    w = wp = None
    if weights == "equal":
        w = wp = rng.uniform(0.2, 1, 8)
    elif weights == "distinct":
        w, wp = rng.uniform(0.2, 1, 8), rng.uniform(0.2, 1, 8)
    lam = landmark_lambda(A, w=w, wp=wp)
    r = path_cv(x, A, lam, w=w, wp=wp)
    fs = _fd(lambda xx: path_cv(xx, A, lam, w=w, wp=wp, grad=False).s, x)
    fz = _fd(lambda xx: path_cv(xx, A, lam, w=w, wp=wp, grad=False).z, x)
    assert np.abs(r.ds_dx - fs).max() <= 1e-7 * np.abs(fs).max()
    assert np.abs(r.dz_dx - fz).max() <= 1e-7 * np.abs(fz).max()


def test_lambda_rule():
    sysm = wl.small_path(10, 6, seed=9)
    A = sysm.landmarks
    d = [msd(A[i + 1], A[i]) for i in range(5)]
    assert abs(landmark_lambda(A) - 2.3 / np.mean(d)) < 1e-9 * landmark_lambda(A)


def test_path_cv_near_landmark_gives_its_index():
    sysm = wl.small_path(15, 9, seed=10, noise_sigma=0.0)
    A = sysm.landmarks
    lam = 50 * landmark_lambda(A)
    for i in (0, 4, 8):
        x, _, _ = wl.rigid_copy(A[i], 100 + i)
        r = path_cv(x, A, lam, grad=False)
        assert abs(r.s - (i + 1)) < 1e-3
        assert r.D[i] < 1e-14
