"""O2: path variables ``s`` and ``z`` over exact landmark distances, FP64.

Test infrastructure only (see ``oracle/__init__.py``).

Paper: Eq. 2 (property-map CV: the ``exp(-lambda D)``-weighted average of
landmark properties ``q_i``), Section 2 (taking the landmark index as the
property gives a CV close to the index of the nearest landmark: the path
variable ``s``), Algorithm 1 (every landmark's rotation, distance and
derivatives are computed each step when no neighbour list is used).

Readings:

* ``q_i = i`` with 1-based landmark indices, so ``1 <= s <= L``.
* ``z = -(1/lambda) ln sum_i exp(-lambda D_i)`` (the distance-from-path
  variable of the path-CV method the paper cites; the paper does not print
  it).  Then ``min D - ln(L)/lambda <= z <= min D``.
* Gradients follow by the chain rule:
  ``ds/dD_i = -lambda p_i (q_i - s)`` and ``dz/dD_i = p_i`` with
  ``p_i = exp(-lambda D_i) / sum_j exp(-lambda D_j)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .msd import normalise_weights, superpose, msd_grad

__all__ = ["PathResult", "path_sz", "path_cv", "landmark_lambda", "default_q"]


def default_q(L: int) -> np.ndarray:
    """Landmark index as the property, 1-based."""
    return np.arange(1, L + 1, dtype=np.float64)


@dataclass
class PathResult:
    s: float
    z: float
    p: np.ndarray          # softmax weights, [L]
    c: np.ndarray          # ds/dD_i, [L]
    D: np.ndarray          # distances used, [L]
    ds_dx: np.ndarray | None = None
    dz_dx: np.ndarray | None = None
    R: np.ndarray | None = None   # optimal rotations (landmark -> x), [L][3][3]


def path_sz(D, lam: float, q=None) -> PathResult:
    """Eq. 2 with the minimum distance factored out of every exponential
    (the ratio and ``z`` are unchanged by a common shift of all ``D_i``)."""
    D = np.asarray(D, dtype=np.float64)
    q = default_q(D.size) if q is None else np.asarray(q, dtype=np.float64)
    m = D.min()
    e = np.exp(-lam * (D - m))
    Z = e.sum()
    s = float((q * e).sum() / Z)
    z = float(m - np.log(Z) / lam)
    p = e / Z
    c = -lam * p * (q - s)
    return PathResult(s, z, p, c, D)


def path_cv(x, A, lam: float, q=None, w=None, wp=None, *, grad: bool = True,
            chunk: int = 512) -> PathResult:
    """Algorithm 1 over all landmarks ``A`` (``[L][n][3]``): exact distances
    (Eq. 3), then ``s``, ``z`` (Eq. 2) and, if ``grad``, their derivatives
    with respect to the raw ``x`` from Eq. 4.

    Landmarks are processed in chunks only to bound memory; pass 1 forms all
    distances, pass 2 (after ``s`` is known) sums ``c_i dD_i/dx``.
    """
    x = np.asarray(x, dtype=np.float64)
    L, n = A.shape[0], A.shape[1]
    w_n = normalise_weights(w, n)
    wp_n = w_n if wp is None else normalise_weights(wp, n)
    D = np.empty(L)
    R = np.empty((L, 3, 3))
    for i0 in range(0, L, chunk):
        sp = superpose(x, A[i0:i0 + chunk], w_n, wp_n)
        D[i0:i0 + chunk] = sp.D
        R[i0:i0 + chunk] = sp.R
    res = path_sz(D, lam, q)
    res.R = R
    if grad:
        gs = np.zeros((n, 3))
        gz = np.zeros((n, 3))
        for i0 in range(0, L, chunk):
            sl = slice(i0, i0 + chunk)
            sp = superpose(x, A[sl], w_n, wp_n)
            gD = msd_grad(x, A[sl], w_n, wp_n, sp=sp)       # [k][n][3]
            gs += np.einsum("i,ija->ja", res.c[sl], gD)
            gz += np.einsum("i,ija->ja", res.p[sl], gD)
        res.ds_dx = gs
        res.dz_dx = gz
    return res


def landmark_lambda(A, factor: float = 2.3, w=None, wp=None) -> float:
    """Sharpness from the mean distance between consecutive landmarks:
    ``lambda = factor / mean_i D(a_i, a_{i+1})`` (the usual path-CV choice;
    the paper does not state its lambda)."""
    A = np.asarray(A, dtype=np.float64)
    d = [superpose(A[i + 1], A[i], w, wp).D for i in range(A.shape[0] - 1)]
    return float(factor / np.mean(d))
