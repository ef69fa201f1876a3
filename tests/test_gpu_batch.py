"""GPU parity of the batched multi-walker engine against the oracle, per walker."""
import numpy as np
import pytest

import workloads as wl
from oracle.path import landmark_lambda, path_cv

pytestmark = pytest.mark.gpu


def _walkers(k, atom_range, landmark_range, stream):
    ws = wl.walkers(n_walkers=k, n_frames=2, atom_range=atom_range, landmark_range=landmark_range, stream=stream)
    lams = [landmark_lambda(w.system.landmarks) for w in ws]
    return ws, lams


@pytest.mark.parametrize("tune", [False, True])
def test_batch_matches_oracle(tune, tmp_path):
    import paper_1801_02362_amd as pcv
    import torch
    from gpu_util import TOL32, check_cv, dev, host, say
    ws, lams = _walkers(9, (20, 700), (3, 90), stream=1)
    say(f"[batch] tune={tune} n={[w.system.n_atoms for w in ws]} L={[w.system.n_landmarks for w in ws]}")
    b = pcv.BatchPathCV([dev(w.system.landmarks, torch.float32) for w in ws], lams, tune=tune,
                        cache_path=str(tmp_path / "tune.json") if tune else None)
    say(f"[batch] plan {b.plan}")
    x = dev(np.concatenate([w.frames[1] for w in ws]), torch.float32)
    for rep in range(2):
        sz, ds, dz = b.eval(x)
        sz, ds, dz = host(sz), host(ds), host(dz)
        for i, w in enumerate(ws):
            ref = path_cv(w.frames[1].astype(np.float64), w.system.landmarks.astype(np.float64), lams[i])
            a0, a1 = b.atom_off[i], b.atom_off[i + 1]
            check_cv(f"walker{i}", TOL32, sz[i], ds[a0:a1], dz[a0:a1], None, ref)
    if tune:
        assert (tmp_path / "tune.json").exists()
    b.close()


def test_batch_equals_single_handles():
    import paper_1801_02362_amd as pcv
    import torch
    from gpu_util import dev, host
    ws, lams = _walkers(5, (100, 2000), (50, 400), stream=2)
    b = pcv.BatchPathCV([dev(w.system.landmarks, torch.float32) for w in ws], lams)
    x = dev(np.concatenate([w.frames[0] for w in ws]), torch.float32)
    sz, ds, _ = b.eval(x)
    sz, ds = host(sz), host(ds)
    for i, w in enumerate(ws):
        cv = pcv.PathCV(dev(w.system.landmarks, torch.float32), lams[i])
        o = cv.eval(dev(w.frames[0], torch.float32))
        assert abs(host(o["sz"])[0] - sz[i, 0]) < 1e-7
        g = host(o["ds_dx"])
        assert np.abs(g - ds[b.atom_off[i]:b.atom_off[i + 1]]).max() <= 1e-5 * np.abs(g).max()
        cv.close()
    b.close()


def test_full_64_walker_batch_every_walker():
    """The 64-walker batch the bench times (atoms U[50, 2000], landmarks
    U[200, 5000], one persistent launch, default plan): every walker's s, z
    and both gradients checked against the oracle in full (the oracle runs
    in a pool of processes while the GPU works)."""
    import paper_1801_02362_amd as pcv
    import torch
    from gpu_util import TOL32, _cv_job, _lam_job, check_cv, dev, host, oracle_pool, say
    ws = wl.walkers(n_walkers=64, n_frames=1)
    order = sorted(range(len(ws)), key=lambda i: -ws[i].system.n_atoms * ws[i].system.n_landmarks)
    with oracle_pool() as pool:
        lam_f = {i: pool.submit(_lam_job, ws[i].system.landmarks) for i in order}
        lams = [lam_f[i].result() for i in range(len(ws))]
        ref_f = {i: pool.submit(_cv_job, (ws[i].frames[0], ws[i].system.landmarks, lams[i])) for i in order}
        b = pcv.BatchPathCV([dev(w.system.landmarks, torch.float32) for w in ws], lams)
        say(f"[batch] full 64 walkers, plan {b.plan}")
        x = dev(np.concatenate([w.frames[0] for w in ws]), torch.float32)
        sz, ds, dz = b.eval(x)
        sz, ds, dz = host(sz), host(ds), host(dz)
        b.close()
        for i, w in enumerate(ws):
            assert 1.0 <= sz[i][0] <= w.system.n_landmarks, f"walker{i}: s out of range"
        assert np.isfinite(ds).all() and np.isfinite(dz).all()
        for i in range(len(ws)):
            ref = ref_f[i].result()
            a0, a1 = b.atom_off[i], b.atom_off[i + 1]
            check_cv(f"walker{i}", TOL32, sz[i], ds[a0:a1], dz[a0:a1], None, ref)
