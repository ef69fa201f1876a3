"""O8: property-map collective variables with several properties per
reference (Eq. 2 with a vector q_i).

Test infrastructure only (see ``oracle/__init__.py``).

Eq. 2 averages a property q_i of the references with the weights
exp(-lambda D_i); Section 2 introduces property maps as the generalisation
of the path variable s (q_i = i).  With P properties per reference
(q_i in R^P) each component is its own CV,

    S_k = sum_i q_ik exp(-lambda D_i) / sum_i exp(-lambda D_i),

with gradient -lambda sum_i p_i (q_ik - S_k) dD_i/dx (p_i the normalised
weights), dD_i/dx from Eq. 4.  Reading: the components share the distances
and the weights; nothing couples them.  Exact distances only (Algorithm 1).
"""
from __future__ import annotations

import numpy as np

from .path import path_cv

__all__ = ["property_map"]


def property_map(x, A, lam: float, Q, w=None):
    """S [P] and dS/dx [P][n][3] for properties ``Q`` [L][P], one component
    at a time through Eq. 2."""
    Q = np.asarray(Q, dtype=np.float64)
    S, G = [], []
    for k in range(Q.shape[1]):
        r = path_cv(x, A, lam, q=Q[:, k], w=w)
        S.append(r.s)
        G.append(r.ds_dx)
    return np.array(S), np.array(G)
