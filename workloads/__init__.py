"""Seeded synthetic inputs for path collective-variable workloads.

This module only draws random numbers and lays them out.  It holds none of
the method's arithmetic (no centring, no superposition, no distances, no
path variables), so both the FP64 oracle and the HIP path can take their
inputs from here without sharing any of the computation they are checked on.

The paper's own molecules (a 24-atom cyclooctane with 521 references and the
304-atom Trp-cage with 2120 references, Section 5) are not available; the
workloads below are path-shaped stand-ins of similar size:

* ``path_22x20``: 22 atoms, 20 landmarks on a 2-waypoint path, FP64.
* ``path_300x500``: 300 atoms, 500 landmarks through 5 random waypoints, FP32, a
  100,000-frame Gaussian random walk (the close-structure workload).
* ``rigid_5000x10000``: 5,000 atoms, 10,000 landmarks = 600 MB of FP32 coordinates,
  a fresh noisy copy of the base conformation every frame (bandwidth case).
* ``walkers``: 64 independent walkers with uniform random atom counts in
  [50, 2000] and landmark counts in [200, 5000].
* ``surrogate_training_walks``: independent walks on the path_300x500 system.
* ``nl_path``: 304 atoms, 2,120 references through 8 waypoints, a walk that
  slides along the path (neighbour-list workload).

Every landmark is a noisy point on a piecewise-linear path between random
conformations (coordinates N(0, 0.3 nm)), then rotated by a Haar-random
rotation and translated by U(-1, 1) nm per axis.  Units are nm throughout.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

ROOT_SEED = 20180107
N_WORKLOADS = 6

__all__ = [
    "ROOT_SEED", "PathSystem", "Walker", "workload_rng", "path_system",
    "random_walk", "path_22x20", "path_300x500", "rigid_5000x10000", "rigid_frames", "walkers",
    "surrogate_training_walks", "nl_path", "small_path", "rigid_copy", "mlp_sizes", "mlp_init", "mlp_unflatten",
    "minibatch_order",
]


# Seed families of the workloads (one SeedSequence child each).
W_PATH_22x20, W_PATH_300x500, W_RIGID, W_WALKERS, W_SURROGATE, W_NL = range(N_WORKLOADS)


def workload_rng(k: int, stream: int = 0) -> np.random.Generator:
    """Independent generator for workload family ``k`` and sub-stream ``stream``."""
    ss = np.random.SeedSequence(ROOT_SEED).spawn(N_WORKLOADS)[k]
    return np.random.default_rng(ss.spawn(stream + 1)[stream])


def _haar(rng: np.random.Generator, count: int) -> np.ndarray:
    """``count`` Haar-distributed proper rotation matrices, shape (count, 3, 3)."""
    return Rotation.random(count, random_state=rng).as_matrix().reshape(count, 3, 3)


@dataclass
class PathSystem:
    """Landmarks of one path plus the data a trajectory starts from.

    ``landmarks`` is AoS ``[L][n][3]`` in ``dtype``; ``waypoints`` are the
    noise-free conformations the path runs through (``[K][n][3]``, FP64).
    """

    n_atoms: int
    n_landmarks: int
    landmarks: np.ndarray
    waypoints: np.ndarray
    dtype: type
    name: str = ""
    meta: dict = field(default_factory=dict)


def path_system(n_atoms: int, n_landmarks: int, n_waypoints: int, *,
                rng: np.random.Generator, dtype=np.float32,
                coord_sigma: float = 0.3, noise_sigma: float = 0.02,
                translate: float = 1.0, name: str = "") -> PathSystem:
    """Landmarks spaced uniformly along a piecewise-linear path.

    Path parameter ``t`` runs over ``[0, n_waypoints - 1]`` at ``n_landmarks``
    uniform points; landmark ``i`` is the linear interpolation between the
    two waypoints around ``t_i``, plus N(0, noise_sigma) noise per coordinate,
    rotated by a Haar rotation and shifted by U(-translate, translate) per axis.
    """
    way = rng.normal(0.0, coord_sigma, size=(n_waypoints, n_atoms, 3))
    t = np.linspace(0.0, n_waypoints - 1.0, n_landmarks)
    seg = np.minimum(np.floor(t).astype(int), n_waypoints - 2)
    frac = (t - seg)[:, None, None]
    base = (1.0 - frac) * way[seg] + frac * way[seg + 1]
    base = base + rng.normal(0.0, noise_sigma, size=base.shape)
    rot = _haar(rng, n_landmarks)
    shift = rng.uniform(-translate, translate, size=(n_landmarks, 1, 3))
    lm = np.einsum("lab,ljb->lja", rot, base) + shift
    return PathSystem(n_atoms, n_landmarks, np.ascontiguousarray(lm.astype(dtype)),
                      way, dtype, name)


def random_walk(start: np.ndarray, n_frames: int, *, rng: np.random.Generator,
                step_sigma: float = 0.005, dtype=np.float32) -> np.ndarray:
    """Gaussian random walk: frame 0 is ``start``; each later frame adds
    N(0, step_sigma) independently to every coordinate.  Shape ``[F][n][3]``."""
    steps = rng.normal(0.0, step_sigma, size=(n_frames,) + start.shape)
    steps[0] = 0.0
    walk = start[None] + np.cumsum(steps, axis=0)
    return np.ascontiguousarray(walk.astype(dtype))


def path_22x20(n_frames: int = 1000) -> tuple[PathSystem, np.ndarray]:
    """22 atoms, 20 landmarks on a 2-waypoint path, FP64, random-walk frames."""
    sysm = path_system(22, 20, 2, rng=workload_rng(W_PATH_22x20, 0), dtype=np.float64, name="path_22x20")
    frames = random_walk(sysm.waypoints[0], n_frames, rng=workload_rng(W_PATH_22x20, 1),
                         dtype=np.float64)
    return sysm, frames


def path_300x500(n_frames: int = 100_000) -> tuple[PathSystem, np.ndarray]:
    """300 atoms, 500 landmarks through 5 waypoints, FP32, random-walk frames."""
    sysm = path_system(300, 500, 5, rng=workload_rng(W_PATH_300x500, 0), dtype=np.float32, name="path_300x500")
    frames = random_walk(sysm.waypoints[0], n_frames, rng=workload_rng(W_PATH_300x500, 1))
    return sysm, frames


def rigid_5000x10000(n_atoms: int = 5000, n_landmarks: int = 10_000) -> tuple[PathSystem, np.ndarray]:
    """Bandwidth workload: landmarks are Haar-rotated, shifted copies of one
    base conformation (N(0, 0.3)) with N(0, 0.05) noise.  Returns the system
    and the base conformation that frames are drawn around."""
    rng = workload_rng(W_RIGID, 0)
    base = rng.normal(0.0, 0.3, size=(n_atoms, 3))
    lm = np.empty((n_landmarks, n_atoms, 3), dtype=np.float32)
    chunk = 1000
    for i0 in range(0, n_landmarks, chunk):
        i1 = min(n_landmarks, i0 + chunk)
        k = i1 - i0
        noisy = base[None] + rng.normal(0.0, 0.05, size=(k, n_atoms, 3))
        rot = _haar(rng, k)
        shift = rng.uniform(-1.0, 1.0, size=(k, 1, 3))
        lm[i0:i1] = (np.einsum("lab,ljb->lja", rot, noisy) + shift).astype(np.float32)
    sysm = PathSystem(n_atoms, n_landmarks, lm, base[None], np.float32, "rigid_5000x10000")
    return sysm, base


def rigid_frames(base: np.ndarray, n_frames: int, seed_stream: int = 1) -> np.ndarray:
    """Fresh ``base + N(0, 0.05)`` frame per step, FP32 ``[F][n][3]``."""
    rng = workload_rng(W_RIGID, seed_stream)
    fr = base[None] + rng.normal(0.0, 0.05, size=(n_frames,) + base.shape)
    return np.ascontiguousarray(fr.astype(np.float32))


@dataclass
class Walker:
    system: PathSystem
    frames: np.ndarray  # [F][n][3] FP32


def walkers(n_walkers: int = 64, n_frames: int = 4, *, atom_range=(50, 2000),
            landmark_range=(200, 5000), stream: int = 0) -> list[Walker]:
    """Independent walkers of uneven size, each a 2-waypoint path with its own
    random-walk frames."""
    rng = workload_rng(W_WALKERS, stream)
    n_w = rng.integers(atom_range[0], atom_range[1] + 1, size=n_walkers)
    l_w = rng.integers(landmark_range[0], landmark_range[1] + 1, size=n_walkers)
    out = []
    for w in range(n_walkers):
        sub = np.random.default_rng(rng.integers(0, 2**63 - 1))
        s = path_system(int(n_w[w]), int(l_w[w]), 2, rng=sub, dtype=np.float32,
                        name=f"walkers.w{w}")
        fr = random_walk(s.waypoints[0], n_frames, rng=sub)
        out.append(Walker(s, fr))
    return out


def nl_path(n_frames: int = 3000, *, steps_per_segment: int = 4000) -> tuple[PathSystem, np.ndarray]:
    """Neighbour-list workload with the sizes of the paper's second system
    (304 atoms, 2120 references; a 50-member list refreshed every 50 steps):
    references through 8 waypoints (as ``path_system``), and a walk that
    slides along the path (one waypoint segment per ``steps_per_segment``
    frames, starting at waypoint 0) with mean-reverting thermal noise
    (x_noise <- 0.99 x_noise + N(0, 0.005) per coordinate and frame, about
    0.035 nm stationary), so the nearest references change over the walk."""
    sysm = path_system(304, 2120, 8, rng=workload_rng(W_NL, 0), dtype=np.float32, name="nl_path")
    rng = workload_rng(W_NL, 1)
    way = sysm.waypoints
    frames = np.empty((n_frames, 304, 3), dtype=np.float32)
    noise = np.zeros((304, 3))
    for t in range(n_frames):
        if t:
            noise = 0.99 * noise + rng.normal(0.0, 0.005, size=noise.shape)
        u = min(t / steps_per_segment, way.shape[0] - 1.0)
        k = min(int(u), way.shape[0] - 2)
        f = u - k
        frames[t] = ((1.0 - f) * way[k] + f * way[k + 1] + noise).astype(np.float32)
    return sysm, frames


def surrogate_training_walks(n_walks: int = 1000, steps: int = 1000,
                        system: PathSystem | None = None) -> np.ndarray:
    """Training frames for the surrogate: ``n_walks`` independent walks of
    ``steps`` frames on the path_300x500 system, each starting at a random landmark's
    waypoint mixture (seeds differ from the path_300x500 test walk).  FP32
    ``[n_walks * steps][n][3]``."""
    if system is None:
        system, _ = path_300x500(n_frames=1)
    rng = workload_rng(W_SURROGATE, 0)
    out = np.empty((n_walks * steps, system.n_atoms, 3), dtype=np.float32)
    kway = system.waypoints.shape[0]
    for w in range(n_walks):
        t = rng.uniform(0.0, kway - 1.0)
        seg = min(int(t), kway - 2)
        f = t - seg
        start = (1 - f) * system.waypoints[seg] + f * system.waypoints[seg + 1]
        out[w * steps:(w + 1) * steps] = random_walk(start, steps, rng=rng)
    return out


def small_path(n_atoms: int, n_landmarks: int, seed: int, *, dtype=np.float64,
               n_waypoints: int = 2, noise_sigma: float = 0.02) -> PathSystem:
    """A small seeded path for unit tests and ragged-shape parity cases."""
    return path_system(n_atoms, n_landmarks, n_waypoints,
                       rng=np.random.default_rng(seed), dtype=dtype,
                       noise_sigma=noise_sigma, name=f"small{n_atoms}x{n_landmarks}")


def rigid_copy(x: np.ndarray, seed: int, translate: float = 1.0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """A Haar-rotated, translated copy of ``x`` (``[n][3]``): returns
    ``(copy, rotation, shift)`` with ``copy = x @ rotation.T + shift``."""
    rng = np.random.default_rng(seed)
    rot = _haar(rng, 1)[0]
    shift = rng.uniform(-translate, translate, size=3)
    return x @ rot.T + shift, rot, shift


# ---- surrogate network parameters (random draws and layout only)
def mlp_sizes(n_atoms: int, hidden: int = 512) -> list[int]:
    """Layer widths of the surrogate: 3n -> H -> H -> H -> 2."""
    return [3 * n_atoms, hidden, hidden, hidden, 2]


def mlp_init(sizes: list[int], seed: int) -> np.ndarray:
    """Flat FP32 initial parameters: for each layer W [fan_in][fan_out]
    drawn N(0, 1/fan_in), then a zero bias [fan_out]."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 4, seed]))
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append(rng.normal(0.0, 1.0 / np.sqrt(a), (a, b)).astype(np.float32).ravel())
        parts.append(np.zeros(b, dtype=np.float32))
    return np.concatenate(parts)


def mlp_unflatten(flat: np.ndarray, sizes: list[int]) -> tuple[list[np.ndarray], list[np.ndarray]]:
    """Split a flat parameter array into per-layer W [fan_in][fan_out] and b."""
    W, b, o = [], [], 0
    for a, c in zip(sizes[:-1], sizes[1:]):
        W.append(np.asarray(flat[o:o + a * c]).reshape(a, c))
        o += a * c
        b.append(np.asarray(flat[o:o + c]))
        o += c
    assert o == len(flat)
    return W, b


def minibatch_order(n: int, epoch: int, seed: int = 0) -> np.ndarray:
    """Seeded permutation of n training rows for one epoch."""
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 4, 1000 + seed, epoch])).permutation(n)
