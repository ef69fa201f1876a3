"""Helpers shared by the GPU tests (imported lazily; needs torch with a GPU)."""
import sys

import numpy as np

# FP32 path tolerances: MSD 1e-5 relative, s and z 1e-6 absolute, gradients
# 1e-5 of the largest gradient entry.  FP64 path: 1e-12 / 1e-11 / 1e-10.
TOL32 = dict(msd_rel=1e-5, msd_abs=1e-12, sz=1e-6, grad=1e-5)
TOL64 = dict(msd_rel=1e-12, msd_abs=1e-15, sz=1e-11, grad=1e-10)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def check_cv(name, tol, sz, ds, dz, D, ref, *, grads=True):
    """Compare GPU outputs with an oracle PathResult."""
    s, z = sz
    assert abs(s - ref.s) <= tol["sz"], f"{name}: s {s} vs {ref.s} (|d|={abs(s - ref.s):.3e})"
    assert abs(z - ref.z) <= tol["sz"], f"{name}: z {z} vs {ref.z} (|d|={abs(z - ref.z):.3e})"
    if D is not None:
        err = np.abs(D - ref.D)
        bound = tol["msd_rel"] * np.abs(ref.D) + tol["msd_abs"]
        assert np.all(err <= bound), f"{name}: MSD worst rel {np.max(err / (np.abs(ref.D) + 1e-300)):.3e}"
    if grads:
        for what, g, r in (("ds/dx", ds, ref.ds_dx), ("dz/dx", dz, ref.dz_dx)):
            e = np.abs(g - r).max()
            scale = np.abs(r).max()
            assert e <= tol["grad"] * scale + 1e-12, f"{name}: {what} err {e:.3e} scale {scale:.3e}"


# Oracle jobs for a process pool (spawned children run NumPy only; they
# never touch the GPU).
def _lam_job(lm):
    from oracle.path import landmark_lambda
    return landmark_lambda(lm)


def _cv_job(args):
    from oracle.path import path_cv
    frame, lm, lam = args
    r = path_cv(np.asarray(frame, dtype=np.float64), np.asarray(lm, dtype=np.float64), lam)
    return r


def oracle_pool():
    """A pool of at most 16 spawned processes for oracle work."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    return cf.ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)),
                                  mp_context=mp.get_context("spawn"))
