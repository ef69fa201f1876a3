"""Pins of the metadynamics-bias oracle (oracle/bias.py): closed forms of the
Hermite basis, exact reproduction of bicubic polynomials, exactness at grid
nodes, the interpolation error bound against the direct hill sum, finite
differences of every derivative, and the chain rule through the path
variables."""
import numpy as np
import pytest

import workloads as wl
from oracle import bias
from oracle.path import landmark_lambda, path_cv


def _grid(ns=41, nz=31, **kw):
    p = dict(s_min=0.5, s_max=6.5, ns=ns, z_min=-0.2, z_max=0.4, nz=nz, height=1.3, sigma_s=0.4, sigma_z=0.05)
    p.update(kw)
    return bias.Grid(**p)


def test_hermite_basis_closed_forms():
    h, d = bias.hermite_basis(0.0)
    assert h == (1.0, 0.0, 0.0, 0.0) and d == (0.0, 1.0, 0.0, 0.0)
    h, d = bias.hermite_basis(1.0)
    assert h == (0.0, 0.0, 1.0, 0.0) and d == (0.0, 0.0, 0.0, 1.0)
    for t in np.linspace(0, 1, 11):
        h, _ = bias.hermite_basis(t)
        assert abs(h[0] + h[2] - 1.0) < 1e-15        # values: partition of unity


def test_bicubic_polynomials_are_reproduced_exactly():
    rng = np.random.default_rng(1)
    c = rng.normal(size=(4, 4))
    g = _grid(ns=7, nz=5)
    P = lambda s, z: sum(c[a, b] * s ** a * z ** b for a in range(4) for b in range(4))
    Ps = lambda s, z: sum(a * c[a, b] * s ** (a - 1) * z ** b for a in range(1, 4) for b in range(4))
    Pz = lambda s, z: sum(b * c[a, b] * s ** a * z ** (b - 1) for a in range(4) for b in range(1, 4))
    Psz = lambda s, z: sum(a * b * c[a, b] * s ** (a - 1) * z ** (b - 1) for a in range(1, 4) for b in range(1, 4))
    for i in range(g.ns):
        for j in range(g.nz):
            s, z = g.s_min + i * g.hs, g.z_min + j * g.hz
            g.data[:, i, j] = (P(s, z), Ps(s, z), Pz(s, z), Psz(s, z))
    for s, z in zip(rng.uniform(g.s_min, g.s_max, 40), rng.uniform(g.z_min, g.z_max, 40)):
        V, Vs, Vz, ok = bias.interpolate(g, s, z)
        assert ok
        assert abs(V - P(s, z)) < 1e-10 * (1 + abs(P(s, z)))
        assert abs(Vs - Ps(s, z)) < 1e-9 * (1 + abs(Ps(s, z)))
        assert abs(Vz - Pz(s, z)) < 1e-9 * (1 + abs(Pz(s, z)))


def test_hill_derivatives_match_finite_differences():
    cen = [(2.0, 0.1), (2.7, 0.05), (3.1, 0.2)]
    f = lambda s, z: bias.hill_sum(s, z, cen, 1.3, 0.4, 0.05)
    s, z, h = 2.4, 0.12, 1e-6
    V, Vs, Vz, Vsz = f(s, z)
    assert abs(Vs - (f(s + h, z)[0] - f(s - h, z)[0]) / (2 * h)) < 1e-7
    assert abs(Vz - (f(s, z + h)[0] - f(s, z - h)[0]) / (2 * h)) < 1e-5
    assert abs(Vsz - (f(s, z + h)[1] - f(s, z - h)[1]) / (2 * h)) < 1e-4


def test_nodes_hold_the_exact_hill_sum():
    g = _grid(ns=13, nz=11)
    cen = [(2.0, 0.1), (4.4, -0.05), (3.3, 0.3)]
    for s0, z0 in cen:
        bias.deposit(g, s0, z0)
    for i in (0, 3, 7, 12):
        for j in (0, 5, 10):
            s, z = min(g.s_min + i * g.hs, g.s_max), min(g.z_min + j * g.hz, g.z_max)
            V, Vs, Vz, ok = bias.interpolate(g, s, z)
            ref = bias.hill_sum(s, z, cen, g.height, g.sigma_s, g.sigma_z)
            assert ok and abs(V - ref[0]) < 1e-12 and abs(Vs - ref[1]) < 1e-10 and abs(Vz - ref[2]) < 1e-9


def test_fine_grid_is_within_the_hermite_error_bound():
    # grid step sigma / 8 in both CVs: cubic Hermite error <= h^4 max|f''''| / 384 per direction
    g = _grid(ns=121, nz=97, s_min=1.0, s_max=1.0 + 120 * 0.05, z_min=-0.2, z_max=-0.2 + 96 * 0.00625)
    cen = [(3.0, 0.1), (3.5, 0.15)]
    for s0, z0 in cen:
        bias.deposit(g, s0, z0)
    rng = np.random.default_rng(3)
    worst = 0.0
    for s, z in zip(rng.uniform(2.0, 4.5, 60), rng.uniform(0.0, 0.25, 60)):
        V, _, _, _ = bias.interpolate(g, s, z)
        worst = max(worst, abs(V - bias.hill_sum(s, z, cen, g.height, g.sigma_s, g.sigma_z)[0]))
    bound = 2 * 2 * g.height * 3 * (1 / 8) ** 4 / 384     # two hills, two directions, max|f''''| <= 3 w / sigma^4
    assert worst <= bound


def test_interpolant_derivatives_match_its_finite_differences():
    g = _grid(ns=21, nz=17)
    for s0, z0 in [(2.0, 0.1), (3.0, 0.0)]:
        bias.deposit(g, s0, z0)
    s, z, h = 2.37, 0.083, 1e-6
    V, Vs, Vz, _ = bias.interpolate(g, s, z)
    fs = (bias.interpolate(g, s + h, z)[0] - bias.interpolate(g, s - h, z)[0]) / (2 * h)
    fz = (bias.interpolate(g, s, z + h)[0] - bias.interpolate(g, s, z - h)[0]) / (2 * h)
    assert abs(Vs - fs) < 1e-6 and abs(Vz - fz) < 1e-5


def test_out_of_range_is_zero():
    g = _grid()
    bias.deposit(g, 3.0, 0.1)
    for s, z in [(0.4, 0.1), (6.6, 0.1), (3.0, -0.21), (3.0, 0.41)]:
        V, Vs, Vz, ok = bias.interpolate(g, s, z)
        assert (V, Vs, Vz, ok) == (0.0, 0.0, 0.0, False)


def test_bias_gradient_is_the_chain_rule_through_the_path_variables():
    sp = wl.small_path(9, 6, 21, dtype=np.float64)
    lam = landmark_lambda(sp.landmarks)
    x = sp.waypoints[1] + np.random.default_rng(4).normal(0, 0.03, (9, 3))
    r = path_cv(x, sp.landmarks, lam)
    g = _grid(s_min=r.s - 3, s_max=r.s + 3, z_min=r.z - 0.3, z_max=r.z + 0.3, ns=61, nz=61,
              sigma_s=0.5, sigma_z=0.05)
    for s0, z0 in [(r.s - 0.2, r.z + 0.01), (r.s + 0.3, r.z - 0.02)]:
        bias.deposit(g, s0, z0)
    V, Vs, Vz, ok, grad = bias.bias_gradient(g, r.s, r.z, r.ds_dx, r.dz_dx)
    assert ok

    def energy(xx):
        rr = path_cv(xx, sp.landmarks, lam, grad=False)
        return bias.interpolate(g, rr.s, rr.z)[0]

    h = 1e-6
    fd = np.zeros_like(x)
    for k in range(9):
        for d in range(3):
            xp = x.copy(); xp[k, d] += h
            xm = x.copy(); xm[k, d] -= h
            fd[k, d] = (energy(xp) - energy(xm)) / (2 * h)
    assert np.allclose(grad, fd, atol=1e-6 * max(1.0, np.abs(fd).max()))
