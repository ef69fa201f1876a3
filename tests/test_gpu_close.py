"""GPU parity of Algorithm 2 (floating close structure, Eq. 5 / Eq. 6) against
the FP64 oracle state machine, frame by frame along a random walk."""
import copy

import numpy as np
import pytest

import workloads as wl
from oracle.close import CloseStructure
from oracle.path import landmark_lambda, path_cv
from oracle.msd import superpose

pytestmark = pytest.mark.gpu


def _walk(torch, lm, frames, lam, eps, *, dtype, tol, name, every=1, plan=None):
    import paper_1801_02362_amd as pcv
    from gpu_util import check_cv, dev, host, say
    say(f"[close] {name}: L={lm.shape[0]} n={lm.shape[1]} frames={len(frames)} eps={eps} plan={plan}")
    cv = pcv.PathCV(dev(lm, dtype), lam, eps=eps)
    if plan is not None:
        cv.set_plan(**plan)
    orc = CloseStructure(lm.astype(np.float64), lam, eps)
    x = torch.empty(lm.shape[1], 3, dtype=dtype, device="cuda")
    ambiguous = 0
    n_re = 0
    for t, f in enumerate(frames):
        x.copy_(torch.as_tensor(f, dtype=dtype))
        o = cv.eval_close(x, grad=True, msd=True)
        rec = int(host(o["recomputed"])[0])
        force = None
        if orc.y is not None:
            Dxy = float(superpose(f.astype(np.float64), orc.y).D)
            if abs(Dxy - eps) < 1e-6 * abs(eps):
                force = bool(rec)
                ambiguous += 1
        st = orc.step(f.astype(np.float64), force=force)
        assert rec == int(st.recomputed), f"{name}[{t}]: decision gpu={rec} oracle={st.recomputed} D_xy={st.D_xy}"
        n_re += rec
        if t % every == 0 or rec:
            check_cv(f"{name}[{t}]", tol, host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), host(o["msd"]),
                     st.result)
    stats = cv.stats()
    assert stats["recomputes"] == orc.recomputes == n_re
    assert stats["frames"] == len(frames)
    assert stats["expensive_msd"] == orc.expensive_msd
    assert stats["approx_frames"] == len(frames) - n_re
    say(f"[close] {name}: recomputes={n_re} ambiguous={ambiguous}")
    cv.close()
    return n_re


def test_path_300x500_walk_fp32():
    import torch
    from gpu_util import TOL32
    sysm, frames = wl.path_300x500(1500)
    lam = landmark_lambda(sysm.landmarks)
    n_re = _walk(torch, sysm.landmarks, frames, lam, 0.01, dtype=torch.float32, tol=TOL32, name="path_300x500",
                 every=5)
    assert n_re >= 2


def test_path_22x20_walk_fp64():
    import torch
    from gpu_util import TOL64
    sysm, frames = wl.path_22x20(1000)
    lam = landmark_lambda(sysm.landmarks)
    n_re = _walk(torch, sysm.landmarks, frames, lam, 0.01, dtype=torch.float64, tol=TOL64, name="path_22x20")
    assert n_re >= 2


def test_threshold_extremes():
    import torch
    from gpu_util import TOL32
    sysm, frames = wl.path_300x500(40)
    lam = landmark_lambda(sysm.landmarks)
    assert _walk(torch, sysm.landmarks, frames, lam, -1.0, dtype=torch.float32, tol=TOL32, name="eps<0") == 40
    assert _walk(torch, sysm.landmarks, frames, lam, float("inf"), dtype=torch.float32, tol=TOL32,
                 name="eps=inf") == 1


def test_forced_reassignment_and_nonfinite_keep_state():
    import paper_1801_02362_amd as pcv
    import torch
    from gpu_util import dev, host
    sysm, frames = wl.path_300x500(30)
    lam = landmark_lambda(sysm.landmarks)
    cv = pcv.PathCV(dev(sysm.landmarks, torch.float32), lam, eps=0.01)
    x = torch.empty(300, 3, dtype=torch.float32, device="cuda")
    outs = []
    for t in range(20):
        if t == 10:
            bad = torch.as_tensor(frames[t], device="cuda").clone()
            bad[0, 0] = float("inf")
            o = cv.eval_close(bad)
            assert int(host(o["recomputed"])[0]) == -1
            with pytest.raises(pcv.PcvError):
                cv.check()
        x.copy_(torch.as_tensor(frames[t]))
        o = cv.eval_close(x)
        outs.append(host(o["sz"]).copy())
    st = cv.stats()
    assert st["frames"] == 20 and st["recomputes"] == 1
    cv.update_close(x)
    assert cv.stats()["recomputes"] == 2
    cv.force_reassign()
    o = cv.eval_close(x)
    assert int(host(o["recomputed"])[0]) == 1
    ref = path_cv(frames[19].astype(np.float64), sysm.landmarks.astype(np.float64), lam, grad=False)
    assert abs(host(o["sz"])[0] - ref.s) < 1e-6
    cv.close()


# Every engine serves both branches of a close-structure step from one
# launch (the device flag picks the reassignment or the approximate problem).
_CLOSE_PLANS = [dict(engine=1, wg=256, apt=4, team=256), dict(engine=2, wg=512, apt=16, team=64, aptg=8, batch=5),
                dict(engine=3, wg=512, apt=8, team=0, aptg=0, batch=0, items=9),
                dict(engine=4, wg=512, apt=12, team=0, aptg=0, batch=0),
                dict(engine=3, wg=512, apt=16, team=0, aptg=0, batch=0, items=9),
                dict(engine=5, wg=512, apt=8, team=0, aptg=0, batch=0, items=9),
                dict(engine=5, wg=512, apt=12, team=0, aptg=0, batch=0, items=4)]


@pytest.mark.parametrize("plan", _CLOSE_PLANS, ids=["engine1", "engine2", "engine3", "engine4", "engine3_four_blocks",
                                                    "engine5", "engine5_three_blocks"])
def test_close_walk_every_engine(plan):
    import torch
    from gpu_util import TOL32
    s = wl.small_path(700, 40, 61, dtype=np.float32)
    frames = wl.random_walk(s.waypoints[0].astype(np.float64), 30, rng=np.random.default_rng(62), step_sigma=0.01)
    lam = landmark_lambda(s.landmarks)
    n_re = _walk(torch, s.landmarks, frames, lam, 0.002, dtype=torch.float32, tol=TOL32,
                 name=f"close_{plan['engine']}", plan=plan)
    assert 2 <= n_re < len(frames)


def test_many_work_items_close_and_exact():
    """1,300 work items (one landmark each): more slots than one pass of the
    merges' slot loops holds, so the exact merge reads headers beyond its
    256 threads, and the one-pass close merge sums item headers and item G
    sums beyond the 256 slots wave 0 reads ahead and partials beyond the
    twelve items per wave it prefetches.  Close walk and Algorithm 1 with
    the same plan against the oracle."""
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, check_cv, dev, host
    s = wl.small_path(300, 1300, 71, dtype=np.float32)
    frames = wl.random_walk(s.waypoints[0].astype(np.float64), 20, rng=np.random.default_rng(72), step_sigma=0.01)
    lam = landmark_lambda(s.landmarks)
    plan = dict(engine=4, wg=512, apt=8, team=0, aptg=0, batch=1, items=1300)
    n_re = _walk(torch, s.landmarks, frames, lam, 0.002, dtype=torch.float32, tol=TOL32, name="many_items", plan=plan)
    assert 2 <= n_re < len(frames)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), lam)
    cv.set_plan(**plan)
    assert cv.plan["items"] == 1300
    for t in range(0, len(frames), 7):
        o = cv.eval(dev(frames[t], torch.float32), msd=True)
        ref = path_cv(frames[t].astype(np.float64), s.landmarks.astype(np.float64), lam)
        check_cv(f"many_items_exact[{t}]", TOL32, host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), host(o["msd"]), ref)
    cv.close()
