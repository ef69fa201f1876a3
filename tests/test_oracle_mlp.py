"""Pins of the surrogate oracle (oracle/mlp.py) against facts it does not
produce itself: exact BF16 neighbours, closed forms of SiLU and Adam,
central finite differences, and the rigid-motion invariances that any
function of an aligned structure must have."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp
from oracle.msd import superpose


def _net(sizes, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    W = [rng.normal(0, scale / np.sqrt(a), (a, b)) for a, b in zip(sizes[:-1], sizes[1:])]
    b = [rng.normal(0, 0.1, (n,)) for n in sizes[1:]]
    return mlp.MLP(W, b, mean=np.array([3.0, 0.01]), std=np.array([1.7, 0.02]))


def _fd(f, x, h=1e-6):
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros(x.shape + np.shape(f(x)))
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy(); xp[i] += h
        xm = x.copy(); xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


def test_bf16_ties_and_exact_values():
    one = 1.0
    assert mlp.bf16(one) == 1.0
    assert mlp.bf16(1 + 2.0 ** -8) == 1.0                  # halfway, ties to even (1.0)
    assert mlp.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6    # halfway, ties to even (1 + 2^-6)
    assert mlp.bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7   # above halfway rounds up
    assert mlp.bf16(-1.5) == -1.5
    assert mlp.bf16(0.0) == 0.0


def test_bf16_is_the_nearest_neighbour():
    rng = np.random.default_rng(1)
    x = rng.normal(0, 10, 2000).astype(np.float32).astype(np.float64)
    r = mlp.bf16(x)
    for v, rv in zip(x, r):
        e = np.floor(np.log2(abs(v)))
        ulp = 2.0 ** (e - 7)
        lo = np.floor(v / ulp) * ulp
        cands = [lo, lo + ulp]
        best = min(cands, key=lambda c: (abs(c - v), (round(c / ulp) % 2)))
        assert rv == best


def test_silu_closed_forms():
    assert mlp.silu(0.0) == 0.0
    assert mlp.silu_grad(0.0) == 0.5
    assert abs(mlp.silu(50.0) - 50.0) < 1e-12
    assert abs(mlp.silu(-50.0)) < 1e-18
    v = np.linspace(-6, 6, 25)
    fd = (mlp.silu(v + 1e-6) - mlp.silu(v - 1e-6)) / 2e-6
    assert np.allclose(mlp.silu_grad(v), fd, atol=1e-9)


def test_input_and_parameter_gradients_match_finite_differences():
    net = _net([6, 5, 5, 4, 2], 2)
    rng = np.random.default_rng(3)
    X = rng.normal(size=(3, 6))
    dy = rng.normal(size=(3, 2))
    cache = mlp.forward(net, X, rounded=False)
    gX = mlp.input_grad(net, cache, dy, rounded=False)
    fd = _fd(lambda Z: float((mlp.forward(net, Z, rounded=False)["y"] * dy).sum()), X)
    assert np.allclose(gX, fd, atol=1e-8)
    dW, db = mlp.param_grads(net, cache, dy, rounded=False)
    for l in range(4):
        def fW(Wl, l=l):
            W = list(net.W); W[l] = Wl
            return float((mlp.forward(mlp.MLP(W, net.b), X, rounded=False)["y"] * dy).sum())
        def fb(bl, l=l):
            b = list(net.b); b[l] = bl
            return float((mlp.forward(mlp.MLP(net.W, b), X, rounded=False)["y"] * dy).sum())
        assert np.allclose(dW[l], _fd(fW, net.W[l]), atol=1e-8)
        assert np.allclose(db[l], _fd(fb, net.b[l]), atol=1e-8)


def test_loss_gradient_closed_form():
    rng = np.random.default_rng(4)
    y, t = rng.normal(size=(5, 2)), rng.normal(size=(5, 2))
    loss, g = mlp.loss_and_grad(y, t)
    assert np.isclose(loss, ((y - t) ** 2).sum() / 5)
    assert np.allclose(g, _fd(lambda Y: mlp.loss_and_grad(Y, t)[0], y), atol=1e-8)


def test_adam_first_steps_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    w0 = np.array([1.0, 1.0, 1.0])
    w1, m, v = mlp.adam_step(w0, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(w1, w0 - 0.01 * np.sign(g))          # bias-corrected first step is lr * sign(g)
    w2, _, _ = mlp.adam_step(w1, g, m, v, 2, lr=0.01, eps=0.0)
    assert np.allclose(w2, w0 - 0.02 * np.sign(g))          # constant gradient: lr * sign(g) again


def test_alignment_is_rigid_motion_invariant():
    s = wl.small_path(12, 2, 5, dtype=np.float64)
    ref = s.landmarks[0]
    x = s.waypoints[1]
    xp, _ = mlp.align(x, ref)
    y, _, _ = wl.rigid_copy(x, 9)
    yp, _ = mlp.align(y, ref)
    assert np.allclose(xp, yp, atol=1e-12)
    rp, _ = mlp.align(ref, ref)
    assert np.allclose(rp, ref - ref.mean(0), atol=1e-12)
    # x' is x moved rigidly: same internal distances
    sp = superpose(xp, x)
    assert sp.D < 1e-24


def test_surrogate_gradient_matches_finite_differences_and_invariances():
    n = 8
    s = wl.small_path(n, 2, 6, dtype=np.float64)
    ref = s.landmarks[0]
    x = s.waypoints[1] + np.random.default_rng(7).normal(0, 0.05, (n, 3))
    net = _net([3 * n, 7, 6, 5, 2], 8, scale=1.0)
    sv, zv, gs, gz = mlp.surrogate(net, x, ref, rounded=False)
    fd = _fd(mlp.surrogate_fd_check_fn(net, ref), x)
    assert np.allclose(gs, fd[..., 0], atol=1e-7)
    assert np.allclose(gz, fd[..., 1], atol=1e-7)
    # translation and rotation invariance of a function of the aligned structure
    for g in (gs, gz):
        assert np.allclose(g.sum(0), 0.0, atol=1e-10)
        assert np.allclose(np.cross(x - x.mean(0), g).sum(0), 0.0, atol=1e-10)
    y, _, _ = wl.rigid_copy(x, 11)
    sv2, zv2, _, _ = mlp.surrogate(net, y, ref, rounded=False)
    assert abs(sv2 - sv) < 1e-10 and abs(zv2 - zv) < 1e-10


def test_rounded_network_stays_close_to_fp64():
    n = 10
    s = wl.small_path(n, 2, 12, dtype=np.float64)
    net = _net([3 * n, 16, 16, 16, 2], 13)
    x = s.waypoints[1]
    a = mlp.surrogate(net, x, s.landmarks[0], rounded=False)
    b = mlp.surrogate(net, x, s.landmarks[0], rounded=True)
    # BF16 operands: ~3 significant digits per product, errors average out over the sums
    assert abs(a[0] - b[0]) < 2e-2 * net.std[0]
    assert abs(a[1] - b[1]) < 2e-2 * net.std[1]
