"""Checkpoint and resume: a handle loaded with another handle's saved state
continues bit for bit as the original (the close structure of Algorithm 2,
its saved rotations, the counters and the neighbour list of Section 2)."""
import numpy as np
import pytest

import workloads as wl
from oracle.path import landmark_lambda

pytestmark = pytest.mark.gpu


def _walk(n, L, T, seed, dtype=np.float32):
    sp = wl.small_path(n, L, seed, dtype=dtype)
    start = sp.landmarks[L // 3].astype(np.float64)
    frames = wl.random_walk(start, T, rng=np.random.default_rng(seed + 1), step_sigma=0.01, dtype=dtype)
    return sp.landmarks, frames


def _run(torch, cv, frames, mode):
    from gpu_util import dev, host
    out = []
    for f in frames:
        x = dev(f, cv.dtype)
        o = cv.eval_close(x) if mode == "close" else cv.eval(x)
        rec = host(o["recomputed"]).copy() if mode == "close" else None
        out.append((host(o["sz"]).copy(), host(o["ds_dx"]).copy(), host(o["dz_dx"]).copy(), rec))
    return out


@pytest.mark.parametrize("mode,M,dtype", [("close", 0, "f32"), ("close", 0, "f64"), ("exact", 8, "f32"),
                                          ("close", 10, "f32")])
def test_resume_continues_bit_for_bit(mode, M, dtype):
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, say
    tdt = torch.float32 if dtype == "f32" else torch.float64
    lm, frames = _walk(40, 60, 40, 17, np.float32 if dtype == "f32" else np.float64)
    lam = landmark_lambda(lm)
    say(f"[state] mode={mode} M={M} dtype={dtype}")
    a = pcv.PathCV(dev(lm, tdt), lam, eps=0.004)
    if M:
        a.set_neighbour_list(M, 5)
    _run(torch, a, frames[:13], mode)
    blob = a.save_state()
    b = pcv.PathCV(dev(lm, tdt), lam, eps=0.004)
    b.load_state(blob)
    if M:
        assert np.array_equal(np.sort(a.neighbour_list()), np.sort(b.neighbour_list()))
    ra = _run(torch, a, frames[13:], mode)
    rb = _run(torch, b, frames[13:], mode)
    for t, (oa, ob) in enumerate(zip(ra, rb)):
        for k in range(3):
            assert np.array_equal(oa[k], ob[k]), f"step {13 + t}: output {k} differs"
        if mode == "close":
            assert np.array_equal(oa[3], ob[3]), f"step {13 + t}: decision differs"
    assert a.stats() == b.stats()
    if mode == "close":
        assert a.stats()["recomputes"] >= 2
    if M:
        assert np.array_equal(a.neighbour_list(), b.neighbour_list())
    a.close()
    b.close()


def test_load_rejects_other_handles_and_bad_bytes():
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    lm, frames = _walk(30, 20, 3, 23)
    a = pcv.PathCV(dev(lm, torch.float32), 50.0)
    a.eval_close(dev(frames[0], torch.float32))
    blob = a.save_state()
    other_n, _ = _walk(31, 20, 1, 23)
    other_lm, _ = _walk(30, 20, 1, 24)
    for L2, blob2 in ((other_n, blob), (other_lm, blob), (lm, blob[:-8]), (lm, b"\0" * len(blob))):
        b = pcv.PathCV(dev(L2, torch.float32), 50.0)
        with pytest.raises(pcv.PcvError):
            b.load_state(blob2)
        b.close()
    b = pcv.PathCV(dev(lm.astype(np.float64), torch.float64), 50.0)
    with pytest.raises(pcv.PcvError):
        b.load_state(blob)
    b.close()
    a.close()
