"""O1: exact MSD after optimal superposition and its derivative, FP64.

Test infrastructure only (see ``oracle/__init__.py``).

Paper: Section 3 (translation is removed by centring both structures on
their weighted centre of mass; the rotation comes from diagonalising a
matrix built from quaternions), Eq. 3 (``D = sum_j w_j |x_j - R a_j|^2``),
Eq. 4 (derivative with a displacement term, a centre-of-mass term weighted
by the alignment weights ``w'`` and a rotation term), Section 3.1 (the two
weight sets).

Readings (where the paper is silent):

* Both weight sets are normalised to sum to one ("mean" square distance).
* The rotation is fitted with the alignment weights ``w'``; ``D`` uses the
  displacement weights ``w``.  The rotation term of Eq. 4 only exists when
  the fitted rotation is not stationary for ``D``, i.e. when ``w != w'``.
* ``R`` maps the reference ``a`` onto ``x``: ``d_j = x_j - R a_j``.
* The "x" of Eq. 4 is an outer product and the final contraction is the
  Frobenius product with ``dR/dx_k``.
* The quaternion matrix is the 4x4 symmetric matrix of Horn / Coutsias
  whose top eigenvector is the optimal unit quaternion; proper rotations
  only (a quaternion cannot encode a reflection).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "normalise_weights", "centre", "correlation", "quaternion_matrix",
    "rotation_from_quaternion", "rotation_jacobian", "Superposition",
    "superpose", "msd", "msd_grad", "rotation_adjoint", "rotation_term",
]


def normalise_weights(w, n: int) -> np.ndarray:
    """Weights as FP64 summing to one; ``None`` means uniform ``1/n``."""
    if w is None:
        return np.full(n, 1.0 / n)
    w = np.asarray(w, dtype=np.float64)
    if w.shape != (n,) or np.any(w < 0) or w.sum() <= 0:
        raise ValueError("weights must be a non-negative length-n vector with a positive sum")
    return w / w.sum()


def centre(x, wp) -> np.ndarray:
    """Subtract the ``w'``-weighted centre of mass (Section 3: translation)."""
    x = np.asarray(x, dtype=np.float64)
    return x - np.einsum("j,...ja->...a", wp, x)[..., None, :]


def correlation(a_c, x_c, wp) -> np.ndarray:
    """``M[a][b] = sum_j w'_j a_j[a] x_j[b]`` for centred structures (3x3, or
    a batch ``[L][3][3]`` when ``a_c`` is ``[L][n][3]``)."""
    return np.einsum("j,...ja,jb->...ab", wp, a_c, x_c)


def quaternion_matrix(M) -> np.ndarray:
    """Symmetric 4x4 matrix whose top eigenpair gives the optimal rotation of
    ``a`` onto ``x`` (Horn / Coutsias form), batched over leading axes."""
    M = np.asarray(M, dtype=np.float64)
    xx, xy, xz = M[..., 0, 0], M[..., 0, 1], M[..., 0, 2]
    yx, yy, yz = M[..., 1, 0], M[..., 1, 1], M[..., 1, 2]
    zx, zy, zz = M[..., 2, 0], M[..., 2, 1], M[..., 2, 2]
    F = np.empty(M.shape[:-2] + (4, 4))
    F[..., 0, 0] = xx + yy + zz
    F[..., 0, 1] = yz - zy
    F[..., 0, 2] = zx - xz
    F[..., 0, 3] = xy - yx
    F[..., 1, 1] = xx - yy - zz
    F[..., 1, 2] = xy + yx
    F[..., 1, 3] = zx + xz
    F[..., 2, 2] = -xx + yy - zz
    F[..., 2, 3] = yz + zy
    F[..., 3, 3] = -xx - yy + zz
    for r in range(4):
        for c in range(r):
            F[..., r, c] = F[..., c, r]
    return F


def rotation_from_quaternion(q) -> np.ndarray:
    """Rotation matrix of a unit quaternion ``(q0, q1, q2, q3)``, batched."""
    q = np.asarray(q, dtype=np.float64)
    q0, q1, q2, q3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3
    R[..., 0, 1] = 2 * (q1 * q2 - q0 * q3)
    R[..., 0, 2] = 2 * (q1 * q3 + q0 * q2)
    R[..., 1, 0] = 2 * (q1 * q2 + q0 * q3)
    R[..., 1, 1] = q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3
    R[..., 1, 2] = 2 * (q2 * q3 - q0 * q1)
    R[..., 2, 0] = 2 * (q1 * q3 - q0 * q2)
    R[..., 2, 1] = 2 * (q2 * q3 + q0 * q1)
    R[..., 2, 2] = q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3
    return R


def rotation_jacobian(q) -> np.ndarray:
    """``dR/dq_m`` for m = 0..3, shape ``[..., 4, 3, 3]`` (R is quadratic in q)."""
    q = np.asarray(q, dtype=np.float64)
    q0, q1, q2, q3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    J = np.empty(q.shape[:-1] + (4, 3, 3))

    def put(m, rows):
        for a in range(3):
            for b in range(3):
                J[..., m, a, b] = 2.0 * rows[a][b]

    put(0, [[q0, -q3, q2], [q3, q0, -q1], [-q2, q1, q0]])
    put(1, [[q1, q2, q3], [q2, -q1, -q0], [q3, q0, -q1]])
    put(2, [[-q2, q1, q0], [q1, q2, q3], [-q0, q3, -q2]])
    put(3, [[-q3, -q0, q1], [q0, -q3, q2], [q1, q2, q3]])
    return J


@dataclass
class Superposition:
    """Optimal superposition of (batched) references ``a`` onto ``x``."""

    x_c: np.ndarray       # centred x, [n][3]
    a_c: np.ndarray       # centred references, [..., n, 3]
    M: np.ndarray         # correlation matrices, [..., 3, 3]
    evals: np.ndarray     # eigenvalues of the quaternion matrix, descending [..., 4]
    evecs: np.ndarray     # matching eigenvectors as columns, [..., 4, 4]
    q: np.ndarray         # top eigenvector (optimal quaternion), [..., 4]
    R: np.ndarray         # rotation mapping a onto x, [..., 3, 3]
    d: np.ndarray         # residuals x_c - R a_c, [..., n, 3]
    D: np.ndarray         # Eq. 3, [...]


def superpose(x, a, w=None, wp=None) -> Superposition:
    """Centre, fit ``R`` with ``w'`` by the quaternion eigenproblem, and form
    the Eq. 3 distance directly as ``sum_j w_j |x_j - R a_j|^2``."""
    x = np.asarray(x, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    n = x.shape[-2]
    w = normalise_weights(w, n)
    wp = w if wp is None else normalise_weights(wp, n)
    x_c = centre(x, wp)
    a_c = centre(a, wp)
    M = correlation(a_c, x_c, wp)
    F = quaternion_matrix(M)
    lam, V = np.linalg.eigh(F)          # ascending
    lam = lam[..., ::-1]
    V = V[..., :, ::-1]
    q = V[..., :, 0]
    R = rotation_from_quaternion(q)
    d = x_c - np.einsum("...ab,...jb->...ja", R, a_c)
    D = np.einsum("j,...ja,...ja->...", w, d, d)
    return Superposition(x_c, a_c, M, lam, V, q, R, d, D)


def msd(x, a, w=None, wp=None) -> float:
    """Eq. 3 for one pair of structures ``[n][3]``."""
    return float(superpose(x, a, w, wp).D)


def rotation_adjoint(sp_evals, sp_evecs, G) -> np.ndarray:
    """Pull a gradient with respect to the rotation back to the correlation
    matrix: returns ``Gamma = d(sum_ab G_ab R_ab)/dM``.

    ``R`` depends on ``M`` only through the top eigenvector ``q`` of the
    quaternion matrix F(M).  First-order eigenvector perturbation gives
    ``dq = sum_{m>0} v_m (v_m . dF q) / (lambda_0 - lambda_m)``; with
    ``g_q = sum_ab G_ab dR_ab/dq`` this is ``mu . dF q`` where
    ``mu = sum_{m>0} v_m (v_m . g_q) / (lambda_0 - lambda_m)``, and since F
    is linear in M, ``Gamma_ab = mu^T F(E_ab) q``.  Batched over leading axes.

    Reading at an exactly degenerate top eigenvalue (zero gap, e.g. a single
    atom or collinear atoms): the sum is a pseudo-inverse, so a zero gap
    contributes nothing (the paper is silent; the rotation is not unique
    there and the distance does not depend on the choice).
    """
    lam = np.asarray(sp_evals)
    V = np.asarray(sp_evecs)
    q = V[..., :, 0]
    J = rotation_jacobian(q)                           # [..., 4, 3, 3]
    g_q = np.einsum("...ab,...mab->...m", G, J)
    mu = 0.0
    for m in range(1, 4):
        v = V[..., :, m]
        gap = lam[..., 0] - lam[..., m]
        num = np.einsum("...k,...k->...", v, g_q)
        coef = np.divide(num, gap, out=np.zeros(np.broadcast(num, gap).shape), where=gap > 0)
        mu = mu + v * coef[..., None]
    Gamma = np.empty(G.shape)
    for a in range(3):
        for b in range(3):
            E = np.zeros((3, 3))
            E[a, b] = 1.0
            FE = quaternion_matrix(E)
            Gamma[..., a, b] = np.einsum("...k,kl,...l->...", mu, FE, q)
    return Gamma


def rotation_term(Gamma, a_c, wp) -> np.ndarray:
    """Contribution of ``Gamma = dL/dM`` to ``dL/dx_k``: ``M`` depends on ``x_k``
    through ``w'_k a_k x_k^T`` (the centring part vanishes because ``a_c`` is
    centred with ``w'``).  Returns ``[..., n, 3]``."""
    return wp[:, None] * np.einsum("...ac,...ka->...kc", Gamma, a_c)


def msd_grad(x, a, w=None, wp=None, *, sp: Superposition | None = None) -> np.ndarray:
    """Eq. 4: ``dD/dx_k`` with respect to the raw (uncentred) ``x``.

    Three terms: the displacement ``2 w_k d_k``; the centre-of-mass term
    ``-2 w'_k sum_j w_j d_j``; and the rotation term, the Frobenius product
    of ``dD/dR = -2 sum_j w_j d_j a_j^T`` with ``dR/dx_k``.  For ``w = w'``
    the last two vanish (both structures are centred with the same weights,
    and ``R`` is stationary for ``D``).
    """
    n = np.asarray(x).shape[-2]
    w_n = normalise_weights(w, n)
    wp_n = w_n if wp is None else normalise_weights(wp, n)
    if sp is None:
        sp = superpose(x, a, w_n, wp_n)
    d = sp.d
    g = 2.0 * w_n[:, None] * d
    g -= 2.0 * wp_n[:, None] * np.einsum("j,...ja->...a", w_n, d)[..., None, :]
    G = -2.0 * np.einsum("j,...ja,...jb->...ab", w_n, d, sp.a_c)
    Gamma = rotation_adjoint(sp.evals, sp.evecs, G)
    g += rotation_term(Gamma, sp.a_c, wp_n)
    return g
