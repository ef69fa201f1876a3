"""Pins for the FP64 oracle's exact MSD (Eq. 3) and derivative (Eq. 4).

Each check ties the oracle to something other than itself: invariants of a
distance after optimal superposition, brute force over a rotation grid, an
SVD-based superposition (Kabsch), the roots of the quaternion matrix's
characteristic polynomial from NumPy, and central finite differences.
"""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

import workloads as wl
from oracle.msd import (centre, msd, msd_grad, normalise_weights, quaternion_matrix,
                        rotation_adjoint, superpose)


def _pair(n, seed, noise=0.1):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 0.3, (n, 3))
    a = x + rng.normal(0, noise, (n, 3))
    a, _, _ = wl.rigid_copy(a, seed + 1000)
    return x, a


def _kabsch(x, a, w):
    """Weighted superposition by SVD with the determinant fix (proper rotations)."""
    xc = x - w @ x
    ac = a - w @ a
    H = (ac * w[:, None]).T @ xc
    U, S, Vt = np.linalg.svd(H)
    dfix = np.sign(np.linalg.det(Vt.T @ U.T))
    Dm = np.diag([1.0, 1.0, dfix])
    R = Vt.T @ Dm @ U.T
    d = xc - ac @ R.T
    return float(np.sum(w[:, None] * d * d)), R


@pytest.mark.parametrize("n,seed", [(4, 1), (7, 2), (22, 3), (300, 4)])
def test_rigid_copy_has_zero_distance(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 0.3, (n, 3))
    y, _, _ = wl.rigid_copy(x, seed)
    assert msd(y, x) < 1e-14
    assert msd(x, y) < 1e-14
    w = rng.uniform(0.1, 1.0, n)
    assert msd(y, x, w, w) < 1e-14


@pytest.mark.parametrize("n,seed", [(5, 11), (22, 12), (120, 13)])
def test_symmetry(n, seed):
    x, a = _pair(n, seed)
    assert abs(msd(x, a) - msd(a, x)) < 1e-15
    w = np.random.default_rng(seed).uniform(0.2, 1.0, n)
    assert abs(msd(x, a, w, w) - msd(a, x, w, w)) < 1e-15


@pytest.mark.parametrize("n,seed", [(4, 21), (5, 22), (9, 23), (64, 24)])
def test_matches_svd_superposition(n, seed):
    x, a = _pair(n, seed, noise=0.2)
    for w in (None, np.random.default_rng(seed).uniform(0.1, 1.0, n)):
        wn = normalise_weights(w, n)
        sp = superpose(x, a, wn, wn)
        Dk, Rk = _kabsch(x, a, wn)
        assert abs(float(sp.D) - Dk) < 1e-13
        assert np.abs(sp.R - Rk).max() < 1e-9


@pytest.mark.parametrize("n,seed", [(5, 25), (30, 26)])
def test_two_weight_sets_match_alignment_superposition(n, seed):
    """w != w': centring and rotation by the alignment weights (an SVD fit
    under w'), then the distance by the displacement weights w."""
    x, a = _pair(n, seed, noise=0.2)
    rng = np.random.default_rng(seed)
    w, wp = normalise_weights(rng.uniform(0.0, 1.0, n), n), normalise_weights(rng.uniform(0.2, 1.0, n), n)
    sp = superpose(x, a, w, wp)
    _, Rk = _kabsch(x, a, wp)
    d = (x - wp @ x) - (a - wp @ a) @ Rk.T
    assert abs(float(sp.D) - float(np.sum(w[:, None] * d * d))) < 1e-13
    assert float(sp.D) > float(superpose(x, a, w, w).D) - 1e-15   # w's own fit is the minimum


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_top_eigenvalue_is_largest_characteristic_root(seed):
    n = 10
    x, a = _pair(n, seed)
    sp = superpose(x, a)
    F = quaternion_matrix(sp.M)
    roots = np.roots(np.poly(F))
    lam0 = float(np.max(roots.real))
    assert abs(lam0 - sp.evals[0]) < 1e-13
    w = np.full(n, 1.0 / n)
    Gx = np.sum(w[:, None] * sp.x_c ** 2)
    Ga = np.sum(w[:, None] * sp.a_c ** 2)
    assert abs((Gx + Ga - 2 * lam0) - float(sp.D)) < 1e-13


def _grid_quaternions(m):
    g = np.arange(-m, m + 1, dtype=np.float64)
    q = np.stack(np.meshgrid(g, g, g, g, indexing="ij"), -1).reshape(-1, 4)
    q = q[(q[:, 0] > 0) | ((q[:, 0] == 0) & (np.linalg.norm(q, axis=1) > 0))]
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


@pytest.mark.parametrize("n,seed", [(4, 41), (5, 42), (6, 43)])
def test_brute_force_rotation_grid(n, seed):
    """No rotation of a fine SO(3) grid beats the oracle's optimum, the best
    grid rotation lies near it, and local polishing from the best grid
    points reproduces the oracle's distance and rotation."""
    x, a = _pair(n, seed, noise=0.25)
    sp = superpose(x, a)
    w = np.full(n, 1.0 / n)
    xc, ac = sp.x_c, sp.a_c
    q = _grid_quaternions(14)
    Rg = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()        # scalar-last for scipy
    d = xc[None] - np.einsum("gab,jb->gja", Rg, ac)
    Dg = np.einsum("j,gja,gja->g", w, d, d)
    assert Dg.min() >= float(sp.D) - 1e-14
    best = np.argsort(Dg)[:8]
    ang = Rotation.from_matrix(Rg[best[0]] @ sp.R.T).magnitude()
    assert ang < 0.3

    def f(rv):
        R = Rotation.from_rotvec(rv).as_matrix()
        dd = xc - ac @ R.T
        return float(np.sum(w[:, None] * dd * dd))

    polished = [minimize(f, Rotation.from_matrix(Rg[b]).as_rotvec(), method="BFGS",
                         options={"gtol": 1e-13}) for b in best]
    top = min(polished, key=lambda r: r.fun)
    assert abs(top.fun - float(sp.D)) < 1e-10
    Rp = Rotation.from_rotvec(top.x).as_matrix()
    assert np.abs(Rp - sp.R).max() < 1e-5


def test_mirror_image_is_not_superposable():
    rng = np.random.default_rng(51)
    x = rng.normal(0, 0.3, (8, 3))
    y = x.copy()
    y[:, 2] *= -1.0
    D = msd(x, y)
    assert D > 1e-3
    Dk, _ = _kabsch(x, y, np.full(8, 1 / 8))
    assert abs(D - Dk) < 1e-13


def _fd(fun, x, h=1e-6):
    g = np.zeros_like(x)
    for k in range(x.shape[0]):
        for c in range(3):
            xp = x.copy(); xp[k, c] += h
            xm = x.copy(); xm[k, c] -= h
            g[k, c] = (fun(xp) - fun(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("case", ["uniform", "equal_weights", "distinct_weights"])
def test_gradient_matches_finite_differences(case):
    n = 9
    x, a = _pair(n, 61, noise=0.2)
    rng = np.random.default_rng(62)
    if case == "uniform":
        w = wp = None
    elif case == "equal_weights":
        w = wp = rng.uniform(0.2, 1.0, n)
    else:
        w, wp = rng.uniform(0.2, 1.0, n), rng.uniform(0.2, 1.0, n)
    g = msd_grad(x, a, w, wp)
    fd = _fd(lambda xx: msd(xx, a, w, wp), x)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max()
    # The distance and gradient are translation invariant.
    assert np.abs(g.sum(axis=0)).max() < 1e-13


def test_gradient_terms_vanish_for_equal_weights():
    """For w = w' the centre-of-mass and rotation terms of Eq. 4 are zero."""
    n = 12
    x, a = _pair(n, 71, noise=0.2)
    w = np.random.default_rng(72).uniform(0.2, 1.0, n)
    wn = normalise_weights(w, n)
    sp = superpose(x, a, wn, wn)
    com = 2.0 * wn[:, None] * (wn @ sp.d)[None]
    G = -2.0 * np.einsum("j,ja,jb->ab", wn, sp.d, sp.a_c)
    Gamma = rotation_adjoint(sp.evals, sp.evecs, G)
    assert np.abs(com).max() < 1e-14
    assert np.abs(Gamma).max() < 1e-13


def test_distinct_weights_rotation_term_is_needed():
    """With w != w' the rotation term is not negligible: dropping it breaks
    agreement with finite differences."""
    n = 9
    x, a = _pair(n, 81, noise=0.3)
    rng = np.random.default_rng(82)
    w, wp = rng.uniform(0.2, 1.0, n), rng.uniform(0.2, 1.0, n)
    wn, wpn = normalise_weights(w, n), normalise_weights(wp, n)
    sp = superpose(x, a, wn, wpn)
    g_no_rot = 2.0 * wn[:, None] * sp.d - 2.0 * wpn[:, None] * (wn @ sp.d)[None]
    fd = _fd(lambda xx: msd(xx, a, w, wp), x)
    assert np.abs(g_no_rot - fd).max() > 1e-4 * np.abs(fd).max()


def test_centre_uses_alignment_weights():
    rng = np.random.default_rng(91)
    x = rng.normal(0, 1, (6, 3)) + 5.0
    wp = normalise_weights(rng.uniform(0.1, 1, 6), 6)
    xc = centre(x, wp)
    assert np.abs(wp @ xc).max() < 1e-14
