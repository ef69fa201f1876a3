"""O3: floating close structure (Algorithm 2, Eq. 5, Eq. 6), FP64.

Test infrastructure only (see ``oracle/__init__.py``).

Paper: Section 3.2.  The state is a close structure ``y`` and one saved
rotation ``R_{a_i y}`` per landmark.  Every step computes the exact
superposition of ``y`` onto the current structure ``x`` (``R_xy``, ``D_xy``
and the derivative of ``R_xy``).  If ``D_xy`` exceeds the threshold
``epsilon`` the close structure is reassigned (``y <- x``) and every
landmark is superposed exactly, saving the new rotations; otherwise the
landmark rotations are approximated by the product ``R_xy R_{a_i y}``
(Eq. 5) and the derivative follows Eq. 6.

Readings:

* ``R_{a_i y}`` maps landmark ``a_i`` into ``y``'s frame and ``R_xy`` maps
  ``y``'s frame onto ``x``; only then is the product a rotation of ``a_i``
  onto ``x`` (the paper's subscript order is not consistent).
* The comparison is strict: ``D_xy == epsilon`` keeps the close structure.
* The first step has no close structure; it runs the exact pass and counts
  as a reassignment ("at the beginning we start as usual").
* A reassignment step returns the exact distances and derivatives.
* ``dR_xy/dx`` (which the paper leaves to the exact-derivative machinery)
  is the first-order eigenvector perturbation of the quaternion eigenproblem
  of ``y`` onto ``x``; see ``oracle.msd.rotation_adjoint``.
* Without a neighbour list both branches loop over all landmarks.
* ``expensive_msd`` counts exact superpositions: one for ``D_xy`` on every
  step that has a close structure, plus ``L`` per reassignment (Section 6.2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .msd import normalise_weights, centre, superpose, rotation_adjoint, rotation_term
from .path import PathResult, default_q, path_sz, path_cv

__all__ = ["CloseStep", "CloseStructure", "approx_distances"]


@dataclass
class CloseStep:
    result: PathResult
    recomputed: bool
    D_xy: float           # distance to the close structure (nan on the first step)


def approx_distances(x_c, R_xy, R_save, A_c, w):
    """Eq. 5: ``D~_i = sum_j w_j |x_j - R_xy R_{a_i y} a_ij|^2`` and the
    residuals, for centred ``x_c`` and centred landmarks ``A_c``."""
    B = np.einsum("iab,ijb->ija", R_save, A_c)          # R_{a_i y} a_ij
    d = x_c[None] - np.einsum("ab,ijb->ija", R_xy, B)
    D = np.einsum("j,ija,ija->i", w, d, d)
    return D, d, B


class CloseStructure:
    """Algorithm 2 as a state machine over a trajectory."""

    def __init__(self, A, lam: float, eps: float, q=None, w=None, wp=None):
        self.A = np.asarray(A, dtype=np.float64)
        self.L, self.n = self.A.shape[0], self.A.shape[1]
        self.lam = float(lam)
        self.eps = float(eps)
        self.q = q
        self.w = normalise_weights(w, self.n)
        self.wp = self.w if wp is None else normalise_weights(wp, self.n)
        self.A_c = centre(self.A, self.wp)
        self.y = None          # centred close structure
        self.R_save = None     # [L][3][3], landmark -> y frame
        self.frames = 0
        self.recomputes = 0
        self.expensive_msd = 0

    # -- Algorithm 2, reassignment branch --------------------------------
    def _reassign(self, x) -> PathResult:
        res = path_cv(x, self.A, self.lam, self.q, self.w, self.wp, grad=True)
        self.y = centre(x, self.wp)
        self.R_save = res.R.copy()
        self.recomputes += 1
        self.expensive_msd += self.L
        return res

    # -- Algorithm 2, approximate branch (Eq. 5 and Eq. 6) ---------------
    def _approx(self, x, sp_xy, idx=None) -> PathResult:
        """Eq. 5 / Eq. 6 over all landmarks, or over the subset ``idx``
        (a neighbour list; properties follow their landmarks)."""
        w, wp = self.w, self.wp
        x_c = sp_xy.x_c
        R_save, A_c, q = self.R_save, self.A_c, self.q
        if idx is not None:
            q = (default_q(self.L) if q is None else np.asarray(q, dtype=np.float64))[idx]
            R_save, A_c = R_save[idx], A_c[idx]
        D, d, B = approx_distances(x_c, sp_xy.R, R_save, A_c, w)
        res = path_sz(D, self.lam, q)
        # Eq. 6 for each landmark: displacement + centre-of-mass + rotation terms.
        g = 2.0 * w[None, :, None] * d
        g -= 2.0 * wp[None, :, None] * np.einsum("j,ija->ia", w, d)[:, None, :]
        G = -2.0 * np.einsum("j,ija,ijb->iab", w, d, B)      # dD~_i/dR_xy
        Gamma = rotation_adjoint(sp_xy.evals[None], sp_xy.evecs[None], G)
        g += rotation_term(Gamma, self.y[None], wp)
        res.ds_dx = np.einsum("i,ija->ja", res.c, g)
        res.dz_dx = np.einsum("i,ija->ja", res.p, g)
        res.R = np.einsum("ab,ibc->iac", sp_xy.R, R_save)
        return res

    def step(self, x, force: bool | None = None) -> CloseStep:
        """One step.  ``force`` overrides the ``D_xy > epsilon`` decision
        (used to follow another implementation across a decision that falls
        within rounding of the threshold)."""
        x = np.asarray(x, dtype=np.float64)
        self.frames += 1
        if self.y is None:
            return CloseStep(self._reassign(x), True, float("nan"))
        sp_xy = superpose(x, self.y, self.w, self.wp)       # y onto x
        self.expensive_msd += 1
        D_xy = float(sp_xy.D)
        recompute = (D_xy > self.eps) if force is None else bool(force)
        if recompute:
            return CloseStep(self._reassign(x), True, D_xy)
        return CloseStep(self._approx(x, sp_xy), False, D_xy)
