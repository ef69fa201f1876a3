"""Pins of the neighbour-list oracle (oracle/nl.py): the full list reproduces
Algorithms 1 and 2, the members are the brute-force nearest references of
the last update frame, the exact identities between the list's CV and the
full CV, and the paper's cost averages (Section 6.2)."""
import numpy as np
import pytest

import workloads as wl
from oracle import cost, nl
from oracle.close import CloseStructure
from oracle.msd import msd
from oracle.path import landmark_lambda, path_cv


def _walk(n=12, L=30, T=24, seed=3, step=0.01, drift=False):
    """Random walk from a waypoint; with ``drift`` it also slides along the
    path (landmark 1 to landmark L over the walk), so the nearest set moves."""
    sp = wl.small_path(n, L, seed, dtype=np.float64)
    rng = np.random.default_rng(seed + 1)
    x0 = sp.landmarks[0] if drift else sp.waypoints[1]
    frames = [x0]
    noise = np.zeros_like(x0)
    for t in range(1, T):
        noise = noise + rng.normal(0, step, x0.shape)
        base = (1 - t / (T - 1)) * sp.landmarks[0] + (t / (T - 1)) * sp.landmarks[-1] if drift else x0
        frames.append(base + noise)
    return sp.landmarks, landmark_lambda(sp.landmarks), np.array(frames)


def test_nearest_orders_by_distance_then_index():
    D = np.array([0.3, 0.1, 0.3, 0.05, 0.1])
    assert list(nl.nearest(D, 5)) == [3, 1, 4, 0, 2]
    assert list(nl.nearest(D, 2)) == [3, 1]


def test_full_list_reproduces_algorithm_1_and_2():
    A, lam, frames = _walk()
    ex = nl.ExactNeighbourList(A, lam, M=A.shape[0], L_nl=5)
    cl = nl.CloseNeighbourList(A, lam, 0.002, M=A.shape[0], L_nl=5)
    cs = CloseStructure(A, lam, 0.002)
    for x in frames:
        r, _ = ex.step(x)
        ref = path_cv(x, A, lam)
        assert abs(r.s - ref.s) < 1e-12 and abs(r.z - ref.z) < 1e-12
        assert np.allclose(r.ds_dx, ref.ds_dx, atol=1e-12, rtol=0)
        st, _ = cl.step(x)
        st2 = cs.step(x)
        assert st.recomputed == st2.recomputed
        assert abs(st.result.s - st2.result.s) < 1e-12 and abs(st.result.z - st2.result.z) < 1e-12
        assert np.allclose(st.result.ds_dx, st2.result.ds_dx, atol=1e-12, rtol=0)


def test_stride_one_is_the_plain_close_structure():
    A, lam, frames = _walk(T=15)
    cl = nl.CloseNeighbourList(A, lam, 0.002, M=4, L_nl=1)
    cs = CloseStructure(A, lam, 0.002)
    for x in frames:
        a, _ = cl.step(x)
        b = cs.step(x)
        assert abs(a.result.s - b.result.s) < 1e-12 and np.allclose(a.result.dz_dx, b.result.dz_dx, atol=1e-12)


def test_members_are_the_brute_force_nearest_of_the_update_frame():
    A, lam, frames = _walk(T=13, drift=True)
    M, L_nl = 6, 4
    q = np.arange(1, A.shape[0] + 1.0)
    ex = nl.ExactNeighbourList(A, lam, M=M, L_nl=L_nl)
    want = None
    for t, x in enumerate(frames):
        r, update = ex.step(x)
        assert update == (t % L_nl == 0)
        if update:
            D = np.array([msd(x, a) for a in A])          # one superposition at a time
            want = sorted(range(len(D)), key=lambda i: (D[i], i))[:M]
            assert list(ex.members) == want
        else:
            ref = path_cv(x, A[want], lam, q[want])
            assert abs(r.s - ref.s) < 1e-12 and abs(r.z - ref.z) < 1e-12
            assert np.allclose(r.ds_dx, ref.ds_dx, atol=1e-12, rtol=0)


def test_list_and_full_cv_differ_by_the_outside_weight_exactly():
    A, lam, frames = _walk()
    x = frames[0]
    M = 5
    ex = nl.ExactNeighbourList(A, lam, M=M, L_nl=100)
    full, _ = ex.step(x)                   # update step: all references
    part, _ = ex.step(x)                   # same structure through the list
    out = np.setdiff1d(np.arange(A.shape[0]), ex.members)
    q = np.arange(1, A.shape[0] + 1.0)
    # s_full - s_list = sum_{outside} p_i (q_i - s_list);  z_list - z_full = -ln(P_list) / lambda
    assert abs((full.s - part.s) - (full.p[out] * (q[out] - part.s)).sum()) < 1e-12
    P_list = full.p[ex.members].sum()
    assert abs((part.z - full.z) + np.log(P_list) / lam) < 1e-12


def test_cost_averages_match_section_6_2():
    A, lam, frames = _walk(T=20)
    N, M, L_nl = A.shape[0], 6, 5
    ex = nl.ExactNeighbourList(A, lam, M=M, L_nl=L_nl)
    for x in frames:
        ex.step(x)
    assert ex.expensive_msd / len(frames) == pytest.approx(cost.expensive_per_step_original(N, M, L_nl), abs=1e-12)
    cl = nl.CloseNeighbourList(A, lam, 0.001, M=M, L_nl=L_nl)
    for x in frames:
        cl.step(x)
    T, R = len(frames), cl.recomputes
    # 1 + N/K with K = T / R, less the first step's missing D(x, y)
    assert cl.expensive_msd / T == pytest.approx(cost.expensive_per_step_close(N, T / R) - 1.0 / T, abs=1e-12)
