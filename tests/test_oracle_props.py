"""Pins of the property-map oracle (oracle/props.py): linearity of Eq. 2 in
the properties, convex-combination bounds, finite differences of every
component's gradient, and rigid-motion invariance."""
import numpy as np

import workloads as wl
from oracle import props
from oracle.path import landmark_lambda


def _case(n=10, L=14, seed=3):
    sp = wl.small_path(n, L, seed, dtype=np.float64)
    lam = landmark_lambda(sp.landmarks)
    x = sp.waypoints[1] + np.random.default_rng(seed).normal(0, 0.03, (n, 3))
    Q = np.random.default_rng(seed + 1).normal(size=(L, 3))
    return sp.landmarks, lam, x, Q


def test_linear_in_the_properties_and_constants_pass_through():
    A, lam, x, Q = _case()
    S, G = props.property_map(x, A, lam, Q)
    a, b, c = 0.7, -1.9, 4.2
    Q2 = np.column_stack([a * Q[:, 0] + b * Q[:, 1] + c, np.full(len(A), c)])
    S2, G2 = props.property_map(x, A, lam, Q2)
    assert abs(S2[0] - (a * S[0] + b * S[1] + c)) < 1e-12
    assert np.allclose(G2[0], a * G[0] + b * G[1], atol=1e-10)
    assert abs(S2[1] - c) < 1e-12 and np.abs(G2[1]).max() < 1e-10


def test_components_are_convex_combinations():
    A, lam, x, Q = _case()
    S, _ = props.property_map(x, A, lam, Q)
    assert np.all(S >= Q.min(axis=0) - 1e-12) and np.all(S <= Q.max(axis=0) + 1e-12)


def test_gradients_match_finite_differences():
    A, lam, x, Q = _case(n=7, L=9)
    S, G = props.property_map(x, A, lam, Q)
    h = 1e-6
    for k in range(7):
        for d in range(3):
            xp = x.copy(); xp[k, d] += h
            xm = x.copy(); xm[k, d] -= h
            fd = (props.property_map(xp, A, lam, Q)[0] - props.property_map(xm, A, lam, Q)[0]) / (2 * h)
            assert np.allclose(G[:, k, d], fd, atol=1e-6 * max(1.0, np.abs(G).max()))


def test_rigid_motion_invariance():
    A, lam, x, Q = _case()
    S, G = props.property_map(x, A, lam, Q)
    y, R, _ = wl.rigid_copy(x, 5)
    S2, G2 = props.property_map(y, A, lam, Q)
    assert np.allclose(S, S2, atol=1e-12)
    assert np.allclose(G2, G @ R.T, atol=1e-9)          # the gradient turns with the structure
