"""Pins for the FP64 oracle's close-structure method (Algorithm 2, Eq. 5, Eq. 6)."""
import copy

import numpy as np
import pytest

import workloads as wl
from oracle.close import CloseStructure
from oracle.path import landmark_lambda, path_cv


@pytest.fixture(scope="module")
def small():
    sysm, frames = wl.path_22x20(300)
    lam = landmark_lambda(sysm.landmarks)
    return sysm, frames, lam


def test_approximate_distance_is_never_below_exact(small):
    sysm, frames, lam = small
    cs = CloseStructure(sysm.landmarks, lam, 0.01)
    for f in frames[:200]:
        st = cs.step(f)
        ex = path_cv(f, sysm.landmarks, lam, grad=False)
        assert np.all(st.result.D >= ex.D - 1e-15)


def test_rigid_motion_of_close_structure_is_exact(small):
    sysm, frames, lam = small
    cs = CloseStructure(sysm.landmarks, lam, 0.01)
    cs.step(frames[10])
    x, _, _ = wl.rigid_copy(frames[10], 77)
    st = cs.step(x)
    assert not st.recomputed and st.D_xy < 1e-14
    ex = path_cv(x, sysm.landmarks, lam)
    assert np.abs(st.result.D - ex.D).max() < 1e-14
    assert abs(st.result.s - ex.s) < 1e-12 and abs(st.result.z - ex.z) < 1e-14
    assert np.abs(st.result.ds_dx - ex.ds_dx).max() < 1e-9 * np.abs(ex.ds_dx).max()
    assert np.abs(st.result.dz_dx - ex.dz_dx).max() < 1e-9 * np.abs(ex.dz_dx).max()


def test_negative_threshold_recomputes_every_step(small):
    sysm, frames, lam = small
    cs = CloseStructure(sysm.landmarks, lam, -1.0)
    for f in frames[:20]:
        st = cs.step(f)
        ex = path_cv(f, sysm.landmarks, lam)
        assert st.recomputed
        assert abs(st.result.s - ex.s) < 1e-13 and abs(st.result.z - ex.z) < 1e-15
        assert np.abs(st.result.ds_dx - ex.ds_dx).max() < 1e-11 * np.abs(ex.ds_dx).max()
    assert cs.recomputes == 20
    assert cs.expensive_msd == 19 + 20 * sysm.n_landmarks


def test_infinite_threshold_recomputes_once(small):
    sysm, frames, lam = small
    cs = CloseStructure(sysm.landmarks, lam, float("inf"))
    for f in frames[:50]:
        cs.step(f)
    assert cs.recomputes == 1 and cs.frames == 50
    assert cs.expensive_msd == 49 + sysm.n_landmarks


def test_reassignment_steps_are_exact(small):
    sysm, frames, lam = small
    cs = CloseStructure(sysm.landmarks, lam, 0.002)
    n_re = 0
    for f in frames[:300]:
        st = cs.step(f)
        if st.recomputed:
            n_re += 1
            ex = path_cv(f, sysm.landmarks, lam)
            assert abs(st.result.s - ex.s) < 1e-13
            assert st.D_xy != st.D_xy or st.D_xy > 0.002
        else:
            assert st.D_xy <= 0.002
    assert n_re >= 2


def test_threshold_is_strict(small):
    sysm, frames, lam = small
    cs = CloseStructure(sysm.landmarks, lam, 0.01)
    cs.step(frames[0])
    probe = copy.deepcopy(cs)
    D_xy = probe.step(frames[40]).D_xy
    cs.eps = D_xy
    assert not cs.step(frames[40]).recomputed


def _fd(fun, x, h=1e-6):
    g = np.zeros_like(x)
    for k in range(x.shape[0]):
        for c in range(3):
            xp = x.copy(); xp[k, c] += h
            xm = x.copy(); xm[k, c] -= h
            g[k, c] = (fun(xp) - fun(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("weights", ["uniform", "distinct"])
def test_approximate_gradient_matches_finite_differences(weights):
    """Eq. 6 including the derivative of the close-structure rotation."""
    sysm = wl.small_path(10, 14, seed=21)
    A = sysm.landmarks
    rng = np.random.default_rng(22)
    w = wp = None
    if weights == "distinct":
        w, wp = rng.uniform(0.2, 1, 10), rng.uniform(0.2, 1, 10)
    lam = landmark_lambda(A, w=w, wp=wp)
    y = sysm.waypoints[0] + rng.normal(0, 0.03, (10, 3))
    x = y + rng.normal(0, 0.02, (10, 3))
    cs = CloseStructure(A, lam, 1.0, w=w, wp=wp)
    cs.step(y)

    def run(xx):
        return copy.deepcopy(cs).step(xx, force=False).result

    r = run(x)
    fs = _fd(lambda xx: run(xx).s, x)
    fz = _fd(lambda xx: run(xx).z, x)
    assert np.abs(r.ds_dx - fs).max() <= 1e-7 * np.abs(fs).max()
    assert np.abs(r.dz_dx - fz).max() <= 1e-7 * np.abs(fz).max()


def test_distance_correlation_along_walk():
    """The approximate and exact distances are almost perfectly correlated
    over a trajectory (Section 6.1)."""
    sysm, frames = wl.path_300x500(1500)
    A = sysm.landmarks
    lam = landmark_lambda(A[:60])
    cs = CloseStructure(A[:60], lam, 0.01)
    De, Da = [], []
    for f in frames[::10]:
        st = cs.step(f)
        if not st.recomputed:
            De.append(path_cv(f, A[:60], lam, grad=False).D)
            Da.append(st.result.D)
    De, Da = np.concatenate(De), np.concatenate(Da)
    assert len(De) > 1000
    assert np.corrcoef(De, Da)[0, 1] > 0.99
    assert np.all(Da >= De - 1e-12)
