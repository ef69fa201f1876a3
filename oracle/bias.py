"""O6: the metadynamics bias of Eq. 1 on the path variables (s, z) and the
bias force through ds/dx and dz/dx.

Test infrastructure only (see ``oracle/__init__.py``).

Eq. 1 sums Gaussian hills deposited at earlier CV values.  Readings (the
paper prints one height ``w`` inside the product over CVs and one width):

* a hill deposited at (s_k, z_k) is
  ``w * exp(-(s - s_k)^2 / (2 sigma_s^2) - (z - z_k)^2 / (2 sigma_z^2))``,
  one height per hill and one width per CV (a single sigma is the case
  sigma_s = sigma_z);
* the bias is kept on a grid, as in the paper's runs: every node of a
  regular (s, z) grid holds the exact hill sum and its derivatives
  V, dV/ds, dV/dz, d2V/(ds dz); between nodes the bias is the bicubic
  Hermite interpolant of those four values at the cell's corners (C1
  continuous, exact for bicubic polynomials);
* outside the grid the bias and its derivatives are zero (reported as
  out of range);
* the bias gradient on the atoms is dV/dx_k = dV/ds ds/dx_k + dV/dz dz/dx_k
  (the force is its negative).

Everything is FP64 and plain loops over hills and nodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Grid", "hill_sum", "deposit", "hermite_basis", "interpolate", "bias_gradient"]


def hill_sum(s, z, centres, height, sigma_s, sigma_z):
    """Direct sum of Gaussian hills: (V, dV/ds, dV/dz, d2V/dsdz) at (s, z)."""
    V = Vs = Vz = Vsz = 0.0
    for sk, zk in centres:
        ds = s - sk
        dz = z - zk
        g = height * np.exp(-ds * ds / (2.0 * sigma_s ** 2) - dz * dz / (2.0 * sigma_z ** 2))
        a = -ds / sigma_s ** 2
        b = -dz / sigma_z ** 2
        V += g
        Vs += a * g
        Vz += b * g
        Vsz += a * b * g
    return V, Vs, Vz, Vsz


@dataclass
class Grid:
    """Regular grid: node (i, j) sits at (s_min + i h_s, z_min + j h_z)."""
    s_min: float
    s_max: float
    ns: int
    z_min: float
    z_max: float
    nz: int
    height: float
    sigma_s: float
    sigma_z: float
    data: np.ndarray = field(default=None)   # [4][ns][nz]: V, Vs, Vz, Vsz
    hills: list = field(default_factory=list)

    def __post_init__(self):
        if self.data is None:
            self.data = np.zeros((4, self.ns, self.nz))

    @property
    def hs(self):
        return (self.s_max - self.s_min) / (self.ns - 1)

    @property
    def hz(self):
        return (self.z_max - self.z_min) / (self.nz - 1)


def deposit(g: Grid, s0: float, z0: float) -> None:
    """Add one hill at (s0, z0) to every node (exact values, no cutoff)."""
    g.hills.append((float(s0), float(z0)))
    for i in range(g.ns):
        s = g.s_min + i * g.hs
        for j in range(g.nz):
            z = g.z_min + j * g.hz
            v = hill_sum(s, z, [(s0, z0)], g.height, g.sigma_s, g.sigma_z)
            for c in range(4):
                g.data[c, i, j] += v[c]


def hermite_basis(t: float):
    """Cubic Hermite basis on [0, 1] and its derivatives in t:
    returns ((h00, h10, h01, h11), (h00', h10', h01', h11'))."""
    t2, t3 = t * t, t * t * t
    h = (2 * t3 - 3 * t2 + 1, t3 - 2 * t2 + t, -2 * t3 + 3 * t2, t3 - t2)
    d = (6 * t2 - 6 * t, 3 * t2 - 4 * t + 1, -6 * t2 + 6 * t, 3 * t2 - 2 * t)
    return h, d


def interpolate(g: Grid, s: float, z: float):
    """(V, dV/ds, dV/dz, in_range) of the bicubic Hermite interpolant."""
    if not (g.s_min <= s <= g.s_max and g.z_min <= z <= g.z_max):
        return 0.0, 0.0, 0.0, False
    hs, hz = g.hs, g.hz
    i = min(int(np.floor((s - g.s_min) / hs)), g.ns - 2)
    j = min(int(np.floor((z - g.z_min) / hz)), g.nz - 2)
    t = (s - (g.s_min + i * hs)) / hs
    u = (z - (g.z_min + j * hz)) / hz
    (h0t, h1t, h2t, h3t), (d0t, d1t, d2t, d3t) = hermite_basis(t)
    (h0u, h1u, h2u, h3u), (d0u, d1u, d2u, d3u) = hermite_basis(u)
    # value basis per corner a (0: left/bottom, 1: right/top) and derivative basis
    Ht = ((h0t, h1t), (h2t, h3t))      # [corner][0: value weight, 1: slope weight]
    Dt = ((d0t, d1t), (d2t, d3t))
    Hu = ((h0u, h1u), (h2u, h3u))
    Du = ((d0u, d1u), (d2u, d3u))
    V = Vs = Vz = 0.0
    for a in (0, 1):
        for b in (0, 1):
            f, fs, fz, fsz = (g.data[c, i + a, j + b] for c in range(4))
            # terms: f * A0 B0 + hs fs A1 B0 + hz fz A0 B1 + hs hz fsz A1 B1
            coef = ((f, hz * fz), (hs * fs, hs * hz * fsz))   # [slope-in-s][slope-in-z]
            for p in (0, 1):
                for q in (0, 1):
                    V += coef[p][q] * Ht[a][p] * Hu[b][q]
                    Vs += coef[p][q] * Dt[a][p] / hs * Hu[b][q]
                    Vz += coef[p][q] * Ht[a][p] * Du[b][q] / hz
    return V, Vs, Vz, True


def bias_gradient(g: Grid, s: float, z: float, ds_dx, dz_dx):
    """(V, dV/ds, dV/dz, in_range, dV/dx [n][3]) at the CV values (s, z)."""
    V, Vs, Vz, ok = interpolate(g, s, z)
    grad = Vs * np.asarray(ds_dx, dtype=np.float64) + Vz * np.asarray(dz_dx, dtype=np.float64)
    return V, Vs, Vz, ok, grad
