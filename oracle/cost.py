"""O4: the cost model of Section 6.2 and Amdahl's law (Eq. 7).

Test infrastructure only (see ``oracle/__init__.py``).

Section 6.2 counts expensive distance computations (a full superposition
with the rotation solved from scratch) per simulation step.  Notation here
follows the paper's section: ``N`` references, neighbour list of ``M``
entries refreshed every ``L_nl`` steps (the paper's ``L``), close structure
reassigned every ``K`` steps on average.
"""
from __future__ import annotations

__all__ = ["expensive_per_step_original", "expensive_per_step_close",
           "close_is_faster", "amdahl"]


def expensive_per_step_original(N: float, M: float = 0.0, L_nl: float = 1.0) -> float:
    """Original method: ``M`` per usual step, all ``N`` every ``L_nl`` steps,
    i.e. ``M + (N - M) / L_nl`` on average.  No neighbour list: ``M = 0``,
    ``L_nl = 1`` gives ``N``."""
    return M + (N - M) / L_nl


def expensive_per_step_close(N: float, K: float) -> float:
    """Close-structure method: one (``D(x, y)``) per step plus ``N`` at each
    reassignment, i.e. ``1 + N / K``."""
    return 1.0 + N / K


def close_is_faster(N: float, M: float, L_nl: float, K: float) -> bool:
    """Speed-up condition ``M + (N - M)/L_nl > 1 + N/K``."""
    return expensive_per_step_original(N, M, L_nl) > expensive_per_step_close(N, K)


def amdahl(p: float, s: float) -> float:
    """Eq. 7: whole-run speed-up when a fraction ``p`` is sped up ``s`` times."""
    return 1.0 / ((1.0 - p) + p / s)
