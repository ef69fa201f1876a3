"""O7: neighbour lists with and without the floating close structure.

Test infrastructure only (see ``oracle/__init__.py``).

Section 2 (property-map CVs) introduces the neighbour list: only the ``M``
references closest to the current structure enter the CV, and the list is
refreshed every ``L_nl`` steps.  Section 3.1 counts ``M`` expensive
distances in a usual step and all ``N`` in an update step; Section 3.2 says
that with the close structure the update step does not recompute the
references exactly but selects them by the approximated distance (Eq. 5),
the exact recomputation happening at reassignment.  Section 6.2's averages
(``M + (N - M)/L_nl`` and ``1 + N/K``) follow from that.

Readings (the paper leaves these open):

* steps are counted from 0; step t is an update step when t is a multiple of
  ``L_nl``; an update step evaluates all ``N`` references, its CV uses all of
  them, and then the ``M`` nearest (ties to the lower index) form the list
  for the following steps;
* with the close structure: a reassignment step evaluates all ``N`` exactly
  and its CV uses all of them (as without a list); an update step without
  reassignment evaluates all ``N`` by Eq. 5; other steps evaluate the list
  members by Eq. 5.  The list is chosen only at update steps (by the
  distances of that step: exact if it reassigned, approximate otherwise); a
  reassignment between updates keeps the members and refreshes their saved
  rotations;
* properties follow their references: the list's CV uses q_i of its members.
"""
from __future__ import annotations

import numpy as np

from .close import CloseStructure
from .msd import normalise_weights
from .path import default_q, path_cv

__all__ = ["nearest", "ExactNeighbourList", "CloseNeighbourList"]


def nearest(D, M: int) -> np.ndarray:
    """Indices of the ``M`` smallest distances, nearest first, ties to the
    lower index."""
    D = np.asarray(D, dtype=np.float64)
    order = np.lexsort((np.arange(D.size), D))
    return order[:M]


class ExactNeighbourList:
    """Algorithm 1 with a neighbour list of ``M`` references refreshed every
    ``L_nl`` steps."""

    def __init__(self, A, lam: float, M: int, L_nl: int, q=None, w=None):
        self.A = np.asarray(A, dtype=np.float64)
        self.N = self.A.shape[0]
        self.lam = float(lam)
        self.M, self.L_nl = int(M), int(L_nl)
        self.q = default_q(self.N) if q is None else np.asarray(q, dtype=np.float64)
        self.w = w
        self.t = 0
        self.members = None
        self.expensive_msd = 0

    def step(self, x):
        """Returns (PathResult, update) for structure ``x``."""
        update = self.t % self.L_nl == 0
        if update:
            res = path_cv(x, self.A, self.lam, self.q, self.w)
            self.members = nearest(res.D, self.M)
            self.expensive_msd += self.N
        else:
            idx = self.members
            res = path_cv(x, self.A[idx], self.lam, self.q[idx], self.w)
            self.expensive_msd += self.M
        self.t += 1
        return res, update


class CloseNeighbourList:
    """Algorithm 2 with a neighbour list (selection by the approximated
    distance at update steps, exact recomputation only at reassignment)."""

    def __init__(self, A, lam: float, eps: float, M: int, L_nl: int, q=None, w=None):
        self.cs = CloseStructure(A, lam, eps, q, w)
        self.N = self.cs.L
        self.M, self.L_nl = int(M), int(L_nl)
        self.t = 0
        self.members = None

    def step(self, x, force: bool | None = None):
        """Returns (CloseStep, update).  ``force`` overrides the reassignment
        decision as in ``CloseStructure.step``."""
        from .close import CloseStep
        from .msd import superpose
        cs = self.cs
        x = np.asarray(x, dtype=np.float64)
        update = self.t % self.L_nl == 0
        cs.frames += 1
        if cs.y is None:
            step = CloseStep(cs._reassign(x), True, float("nan"))
        else:
            sp_xy = superpose(x, cs.y, cs.w, cs.wp)
            cs.expensive_msd += 1
            D_xy = float(sp_xy.D)
            recompute = (D_xy > cs.eps) if force is None else bool(force)
            if recompute:
                step = CloseStep(cs._reassign(x), True, D_xy)
            elif update:
                step = CloseStep(cs._approx(x, sp_xy), False, D_xy)
            else:
                step = CloseStep(cs._approx(x, sp_xy, self.members), False, D_xy)
        if update:
            self.members = nearest(step.result.D, self.M)
        self.t += 1
        return step, update

    @property
    def expensive_msd(self):
        return self.cs.expensive_msd

    @property
    def recomputes(self):
        return self.cs.recomputes
