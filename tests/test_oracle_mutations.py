"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins catch each one: a transposed rotation, a wrong sign in the quaternion
matrix, a dropped centre-of-mass term, a wrong sign in ds/dD."""
import numpy as np
import pytest

import oracle.msd as om
import oracle.path as op
import workloads as wl


def _rigid_pin_holds():
    rng = np.random.default_rng(1)
    x = rng.normal(0, 0.3, (9, 3))
    y, _, _ = wl.rigid_copy(x, 2)
    return om.msd(y, x) < 1e-14


def _fd_pin_holds(w, wp):
    rng = np.random.default_rng(3)
    x = rng.normal(0, 0.3, (7, 3))
    a, _, _ = wl.rigid_copy(x + rng.normal(0, 0.2, (7, 3)), 4)
    g = om.msd_grad(x, a, w, wp)
    h = 1e-6
    fd = np.zeros_like(x)
    for k in range(7):
        for c in range(3):
            xp = x.copy(); xp[k, c] += h
            xm = x.copy(); xm[k, c] -= h
            fd[k, c] = (om.msd(xp, a, w, wp) - om.msd(xm, a, w, wp)) / (2 * h)
    return np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max()


def test_unmutated_pins_hold():
    assert _rigid_pin_holds()
    w, wp = np.linspace(0.3, 1, 7), np.linspace(1, 0.4, 7)
    assert _fd_pin_holds(w, wp)


def test_transposed_rotation_is_caught(monkeypatch):
    orig = om.rotation_from_quaternion
    monkeypatch.setattr(om, "rotation_from_quaternion", lambda q: np.swapaxes(orig(q), -1, -2))
    assert not _rigid_pin_holds()


def test_quaternion_matrix_sign_is_caught(monkeypatch):
    orig = om.quaternion_matrix

    def bad(M):
        F = orig(M)
        F[..., 0, 1] *= -1
        F[..., 1, 0] *= -1
        return F

    monkeypatch.setattr(om, "quaternion_matrix", bad)
    assert not _rigid_pin_holds()


def test_dropped_rotation_term_is_caught(monkeypatch):
    monkeypatch.setattr(om, "rotation_term", lambda Gamma, a_c, wp: 0.0 * a_c)
    assert not _fd_pin_holds(np.linspace(0.3, 1, 7), np.linspace(1, 0.4, 7))


def test_wrong_path_gradient_sign_is_caught(monkeypatch):
    orig = op.path_sz

    def bad(D, lam, q=None):
        r = orig(D, lam, q)
        r.c = -r.c
        return r

    monkeypatch.setattr(op, "path_sz", bad)
    sysm = wl.small_path(6, 8, seed=5)
    A = sysm.landmarks
    x = sysm.waypoints[0] + 0.01
    lam = op.landmark_lambda(A)
    r = op.path_cv(x, A, lam)
    h = 1e-6
    xp = x.copy(); xp[2, 1] += h
    xm = x.copy(); xm[2, 1] -= h
    fd = (op.path_cv(xp, A, lam, grad=False).s - op.path_cv(xm, A, lam, grad=False).s) / (2 * h)
    assert abs(r.ds_dx[2, 1] - fd) > 1e-6 * max(1.0, abs(fd))


# ---- surrogate oracle (oracle/mlp.py)
import oracle.mlp as om5


def _surrogate_pins_hold():
    n = 6
    s = wl.small_path(n, 2, 21, dtype=np.float64)
    ref = s.landmarks[0]
    x = s.waypoints[1] + np.random.default_rng(22).normal(0, 0.05, (n, 3))
    rng = np.random.default_rng(23)
    sizes = [3 * n, 5, 5, 4, 2]
    net = om5.MLP([rng.normal(0, 1 / np.sqrt(a), (a, b)) for a, b in zip(sizes[:-1], sizes[1:])],
                  [rng.normal(0, 0.1, (b,)) for b in sizes[1:]])
    _, _, gs, _ = om5.surrogate(net, x, ref, rounded=False)
    f = om5.surrogate_fd_check_fn(net, ref)
    h = 1e-6
    fd = np.zeros_like(x)
    for k in range(n):
        for c in range(3):
            xp = x.copy(); xp[k, c] += h
            xm = x.copy(); xm[k, c] -= h
            fd[k, c] = (f(xp)[0] - f(xm)[0]) / (2 * h)
    return np.abs(gs - fd).max() <= 1e-6 * np.abs(fd).max()


def test_surrogate_pins_hold_unmutated():
    assert _surrogate_pins_hold()


def test_wrong_silu_derivative_is_caught(monkeypatch):
    monkeypatch.setattr(om5, "silu_grad", lambda v: 1.0 / (1.0 + np.exp(-np.asarray(v))))
    assert not _surrogate_pins_hold()


def test_dropped_alignment_rotation_term_is_caught(monkeypatch):
    monkeypatch.setattr(om5, "rotation_term", lambda Gamma, a_c, wp: np.zeros(a_c.shape))
    assert not _surrogate_pins_hold()


def test_untransposed_backward_weight_is_caught(monkeypatch):
    orig = om5.input_grad

    def bad(net, cache, dy, *, rounded=True):
        ds = om5._backward(net, cache, dy, rounded)
        W0 = net.W[0]
        return ds[0] @ np.resize(W0, (W0.shape[1], W0.shape[0]))
    monkeypatch.setattr(om5, "input_grad", bad)
    assert not _surrogate_pins_hold()


# --- metadynamics bias (oracle/bias.py): planted mistakes caught by its pins
import oracle.bias as ob
import test_oracle_bias as tb


def test_bias_swapped_hermite_slope_basis_is_caught(monkeypatch):
    orig = ob.hermite_basis

    def bad(t):
        (h0, h1, h2, h3), (d0, d1, d2, d3) = orig(t)
        return (h0, h3, h2, h1), (d0, d3, d2, d1)

    monkeypatch.setattr(ob, "hermite_basis", bad)
    with pytest.raises(AssertionError):
        tb.test_bicubic_polynomials_are_reproduced_exactly()


def test_bias_wrong_hill_derivative_sign_is_caught(monkeypatch):
    orig = ob.hill_sum

    def bad(s, z, centres, height, sigma_s, sigma_z):
        V, Vs, Vz, Vsz = orig(s, z, centres, height, sigma_s, sigma_z)
        return V, -Vs, Vz, Vsz

    monkeypatch.setattr(ob, "hill_sum", bad)
    with pytest.raises(AssertionError):
        tb.test_hill_derivatives_match_finite_differences()
    with pytest.raises(AssertionError):
        tb.test_fine_grid_is_within_the_hermite_error_bound()


def test_bias_dropped_z_term_in_the_force_is_caught(monkeypatch):
    def bad(g, s, z, ds_dx, dz_dx):
        V, Vs, Vz, ok = ob.interpolate(g, s, z)
        return V, Vs, Vz, ok, Vs * np.asarray(ds_dx, dtype=np.float64)

    monkeypatch.setattr(ob, "bias_gradient", bad)
    with pytest.raises(AssertionError):
        tb.test_bias_gradient_is_the_chain_rule_through_the_path_variables()


# --- neighbour list (oracle/nl.py)
import oracle.nl as onl
import test_oracle_nl as tn


def test_nl_farthest_members_are_caught(monkeypatch):
    orig = onl.nearest
    monkeypatch.setattr(onl, "nearest", lambda D, M: orig(-np.asarray(D), M))
    with pytest.raises(AssertionError):
        tn.test_members_are_the_brute_force_nearest_of_the_update_frame()


def test_nl_stale_list_is_caught(monkeypatch):
    orig = onl.nearest
    calls = []

    def first_only(D, M):          # the list is chosen once and never refreshed
        calls.append(1)
        return orig(D, M) if len(calls) == 1 else first_only.kept
    first_only.kept = None

    def wrapped(D, M):
        r = first_only(D, M)
        if first_only.kept is None:
            first_only.kept = r
        return r

    monkeypatch.setattr(onl, "nearest", wrapped)
    with pytest.raises(AssertionError):
        tn.test_members_are_the_brute_force_nearest_of_the_update_frame()


# --- property maps (oracle/props.py)
import oracle.props as opr
import test_oracle_props as tpr


def test_props_gradient_sign_is_caught(monkeypatch):
    orig = opr.path_cv

    def bad(*a, **k):
        r = orig(*a, **k)
        r.ds_dx = -r.ds_dx
        return r

    monkeypatch.setattr(opr, "path_cv", bad)
    with pytest.raises(AssertionError):
        tpr.test_gradients_match_finite_differences()
