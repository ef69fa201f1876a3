"""GPU parity of the neighbour list (Section 2; with the close structure,
Section 3.2) against the FP64 oracle, step by step along a walk that slides
along the path so that the list changes between updates."""
import numpy as np
import pytest

import workloads as wl
from oracle import nl
from oracle.msd import superpose
from oracle.path import landmark_lambda, path_cv

pytestmark = pytest.mark.gpu


def _sliding_walk(n, L, T, seed, step=0.004):
    sp = wl.small_path(n, L, seed, dtype=np.float32)
    rng = np.random.default_rng(seed + 7)
    noise = np.zeros((n, 3))
    frames = []
    for t in range(T):
        if t:
            noise = noise + rng.normal(0, step, (n, 3))
        u = t / (T - 1)
        frames.append(((1 - u) * sp.landmarks[2] + u * sp.landmarks[-3] + noise).astype(np.float32))
    return sp.landmarks, np.array(frames)


def _check_members(name, gpu_members, D_ref, M):
    """The device's list must be a nearest set for the oracle's distances:
    equal to the oracle's choice except for swaps within rounding."""
    gpu = np.sort(gpu_members)
    assert len(set(gpu.tolist())) == M and gpu.min() >= 0 and gpu.max() < D_ref.size, name
    inside = D_ref[gpu].max()
    outside = np.delete(D_ref, gpu).min() if M < D_ref.size else np.inf
    assert inside <= outside + 1e-5 * max(1.0, abs(outside)), f"{name}: list is not a nearest set"


def test_exact_neighbour_list_walk():
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, check_cv, dev, host, say
    lm, frames = _sliding_walk(40, 60, 31, 5)
    lam = landmark_lambda(lm)
    M, stride = 8, 5
    say(f"[nl] exact list: L=60 n=40 M={M} stride={stride} frames={len(frames)}")
    cv = pcv.PathCV(dev(lm, torch.float32), lam)
    cv.set_neighbour_list(M, stride)
    orc = nl.ExactNeighbourList(lm.astype(np.float64), lam, M, stride)
    x = torch.empty(40, 3, dtype=torch.float32, device="cuda")
    changes = 0
    prev = None
    for t, f in enumerate(frames):
        x.copy_(torch.as_tensor(f))
        o = cv.eval(x)
        ref, update = orc.step(f.astype(np.float64))
        check_cv(f"nl_exact[{t}]", TOL32, host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), None, ref)
        if update:
            members = cv.neighbour_list()
            _check_members(f"nl_exact[{t}]", members, ref.D, M)
            orc.members = members.astype(np.int64)        # follow the device across near-ties
            if prev is not None and set(prev) != set(members):
                changes += 1
            prev = members
    st = cv.stats()
    assert st["exact_evals"] == len(frames)
    assert st["expensive_msd"] == orc.expensive_msd
    assert changes >= 2
    cv.close()


@pytest.mark.parametrize("eps", [0.004, 0.02])
def test_close_structure_neighbour_list_walk(eps):
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, check_cv, dev, host, say
    lm, frames = _sliding_walk(40, 60, 41, 9)
    lam = landmark_lambda(lm)
    M, stride = 10, 4
    say(f"[nl] close list: L=60 n=40 M={M} stride={stride} eps={eps} frames={len(frames)}")
    cv = pcv.PathCV(dev(lm, torch.float32), lam, eps=eps)
    cv.set_neighbour_list(M, stride)
    orc = nl.CloseNeighbourList(lm.astype(np.float64), lam, eps, M, stride)
    x = torch.empty(40, 3, dtype=torch.float32, device="cuda")
    n_re = 0
    for t, f in enumerate(frames):
        x.copy_(torch.as_tensor(f))
        o = cv.eval_close(x)
        rec = int(host(o["recomputed"])[0])
        force = None
        if orc.cs.y is not None:
            Dxy = float(superpose(f.astype(np.float64), orc.cs.y).D)
            if abs(Dxy - eps) < 1e-6 * eps:
                force = bool(rec)
        st, update = orc.step(f.astype(np.float64), force=force)
        assert rec == int(st.recomputed), f"nl_close[{t}]: decision"
        n_re += rec
        check_cv(f"nl_close[{t}]", TOL32, host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), None, st.result)
        if update:
            members = cv.neighbour_list()
            _check_members(f"nl_close[{t}]", members, st.result.D, M)
            orc.members = members.astype(np.int64)
    stats = cv.stats()
    assert stats["recomputes"] == orc.recomputes == n_re
    assert stats["expensive_msd"] == orc.expensive_msd
    assert n_re >= 2
    cv.close()


def test_full_list_equals_no_list():
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    lm, frames = _sliding_walk(30, 20, 6, 3)
    lam = landmark_lambda(lm)
    a = pcv.PathCV(dev(lm, torch.float32), lam)
    b = pcv.PathCV(dev(lm, torch.float32), lam)
    b.set_neighbour_list(20, 3)
    for f in frames:
        x = dev(f, torch.float32)
        oa, ob = a.eval(x), b.eval(x)
        assert np.allclose(host(oa["sz"]), host(ob["sz"]), atol=1e-9)
        assert np.allclose(host(oa["ds_dx"]), host(ob["ds_dx"]), atol=1e-6 * np.abs(host(oa["ds_dx"])).max())
    a.close()
    b.close()


def test_neighbour_list_arguments():
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    lm, frames = _sliding_walk(10, 12, 2, 4)
    cv = pcv.PathCV(dev(lm, torch.float32), 50.0)
    for M, stride in [(13, 1), (-1, 1), (3, 0)]:
        with pytest.raises(pcv.PcvError):
            cv.set_neighbour_list(M, stride)
    cv.set_neighbour_list(3, 2)
    assert sorted(cv.neighbour_list().tolist()) == [0, 1, 2]
    with pytest.raises(pcv.PcvError):
        cv.eval(dev(frames[0], torch.float32), msd=True)
    cv.set_neighbour_list(0, 1)
    assert cv.neighbour_list().size == 0
    cv.eval(dev(frames[0], torch.float32), msd=True)
    cv.close()
    big = np.random.default_rng(1).normal(0, 0.3, (8193, 4, 3)).astype(np.float32)
    cv = pcv.PathCV(dev(big, torch.float32), 50.0)
    with pytest.raises(pcv.PcvError):
        cv.set_neighbour_list(10, 5)
    cv.close()
