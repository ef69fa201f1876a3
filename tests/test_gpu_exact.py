"""GPU parity of Algorithm 1 (exact MSD, s, z, gradients) against the FP64 oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle.path import landmark_lambda, path_cv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _run_exact(torch, lm, frames, lam, *, dtype, tol, name, q=None, w=None, plan=None, use_graph=True):
    import paper_1801_02362_amd as pcv
    from gpu_util import check_cv, dev, host, say
    say(f"[exact] {name}: L={lm.shape[0]} n={lm.shape[1]} frames={len(frames)} plan={plan}")
    cv = pcv.PathCV(dev(lm, dtype), lam, q=q, w=w, use_graph=use_graph)
    if plan is not None:
        cv.set_plan(**plan)
    x = torch.empty(lm.shape[1], 3, dtype=dtype, device="cuda")
    for t, f in enumerate(frames):
        x.copy_(torch.as_tensor(f, dtype=dtype))
        o = cv.eval(x, grad=True, msd=True)
        ref = path_cv(f.astype(np.float64), lm.astype(np.float64), lam, q=q, w=w)
        check_cv(f"{name}[{t}]", tol, host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), host(o["msd"]), ref)
    cv.check()
    st = cv.stats()
    assert st["exact_evals"] == len(frames)
    assert st["expensive_msd"] == len(frames) * lm.shape[0]
    cv.close()


def test_path_22x20_fp64(torch):
    from gpu_util import TOL64
    sysm, frames = wl.path_22x20(1000)
    lam = landmark_lambda(sysm.landmarks)
    _run_exact(torch, sysm.landmarks, frames[::50], lam, dtype=torch.float64, tol=TOL64, name="path_22x20")


def test_rigid_5000x10000_full_size_in_the_bench_configuration(torch):
    """5,000 atoms x 10,000 landmarks (600 MB), the plan the bench times
    (engine 5, one item per CU): every D_i, s, z and both gradients of one
    frame against the oracle."""
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, check_cv, dev, host, say
    sysm, base = wl.rigid_5000x10000(n_atoms=5000, n_landmarks=10000)
    f = wl.rigid_frames(base, 1)[0]
    cv = pcv.PathCV(dev(sysm.landmarks, torch.float32), None)
    say(f"[exact] rigid_5000x10000 full size: plan={cv.plan} lambda={cv.lam:.4f}")
    assert cv.plan["engine"] == 5 and cv.plan["items"] == cv.plan["grid"]
    o = cv.eval(dev(f, torch.float32), msd=True)
    got = host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), host(o["msd"])
    cv.check()
    cv.close()
    ref = path_cv(f.astype(np.float64), sysm.landmarks.astype(np.float64), cv.lam)
    check_cv("rigid_full", TOL32, *got, ref)


def test_path_300x500_fp32_near_and_far_frames(torch):
    from gpu_util import TOL32
    sysm, frames = wl.path_300x500(100_000)
    lam = landmark_lambda(sysm.landmarks)
    pick = [0, 1, 100, 1000, 5000, 20000, 50000, 99999]
    _run_exact(torch, sysm.landmarks, frames[pick], lam, dtype=torch.float32, tol=TOL32, name="path_300x500")


@pytest.mark.parametrize("n,L,seed", [(1, 3, 1), (2, 4, 2), (3, 1, 3), (5, 2, 4), (17, 37, 5), (63, 64, 6),
                                      (64, 65, 7), (65, 129, 8), (257, 33, 9), (1000, 40, 10), (2049, 23, 11),
                                      (5000, 19, 12), (8192, 5, 13)])
def test_ragged_shapes_fp32(torch, n, L, seed):
    from gpu_util import TOL32
    s = wl.small_path(n, L, seed, dtype=np.float32)
    rng = np.random.default_rng(seed)
    frames = (s.waypoints[0] + rng.normal(0, 0.02, (2, n, 3))).astype(np.float32)
    lam = landmark_lambda(s.landmarks) if L > 1 and n > 1 else 100.0
    _run_exact(torch, s.landmarks, frames, lam, dtype=torch.float32, tol=TOL32, name=f"ragged{n}x{L}")


@pytest.mark.parametrize("n,L,seed", [(1, 2, 21), (22, 20, 22), (130, 70, 23), (2048, 9, 24)])
def test_ragged_shapes_fp64(torch, n, L, seed):
    from gpu_util import TOL64
    s = wl.small_path(n, L, seed, dtype=np.float64)
    rng = np.random.default_rng(seed)
    frames = s.waypoints[0] + rng.normal(0, 0.02, (2, n, 3))
    lam = landmark_lambda(s.landmarks) if n > 1 else 100.0
    _run_exact(torch, s.landmarks, frames, lam, dtype=torch.float64, tol=TOL64, name=f"ragged64_{n}x{L}")


def test_weights_and_properties(torch):
    from gpu_util import TOL32
    s = wl.small_path(150, 60, 31, dtype=np.float32)
    rng = np.random.default_rng(32)
    w = rng.uniform(0.1, 2.0, 150)
    q = rng.normal(size=60)
    frames = (s.waypoints[0] + rng.normal(0, 0.02, (2, 150, 3))).astype(np.float32)
    lam = landmark_lambda(s.landmarks, w=w)
    _run_exact(torch, s.landmarks, frames, lam, dtype=torch.float32, tol=TOL32, name="weights", q=q, w=w)


def _plans(n, wg_apt, e2):
    out = []
    for wg, apt in wg_apt:
        ts = 16
        while ts * apt < n:
            ts *= 2
        while ts <= wg:
            out.append(dict(engine=1, wg=wg, apt=apt, team=ts))
            ts *= 4
    n_pad = (n + 63) // 64 * 64
    for ncw, aptc, aptg in e2:
        for g in (16, 32, 64, 64 * ncw):
            if -(-n_pad // g) <= aptc and -(-n_pad // (64 * (7 - ncw))) <= aptg:
                for batch in (1, 5, 13):
                    out.append(dict(engine=2, wg=512, apt=aptc, team=g, aptg=aptg, batch=batch))
    return out


@pytest.mark.parametrize("plan", _plans(300, [(256, 1), (256, 2), (256, 4), (256, 8), (512, 8), (512, 10), (512, 16)],
                                        [(3, 4, 2), (3, 8, 4), (3, 16, 8), (2, 40, 16)]))
def test_every_tiling_matches(torch, plan):
    from gpu_util import TOL32
    sysm, frames = wl.path_300x500(3000)
    lam = landmark_lambda(sysm.landmarks)
    _run_exact(torch, sysm.landmarks, frames[[0, 2999]], lam, dtype=torch.float32, tol=TOL32,
               name="tiling", plan=plan)


# Large-structure engine: each compiled block count, structures that end
# inside a 256-atom block or a 64-atom tile, and item counts from one item
# (the whole landmark range streamed by one workgroup) to one landmark each.
_E3_CASES = [(n, bpw, items) for n, bpws in ((100, (1, 2, 3)), (700, (1, 2, 3, 4)), (1800, (2, 3)), (1793, (2, 3)),
                                            (3000, (2, 3)), (3584, (2, 3, 4)), (5000, (3, 4)), (5376, (3, 4)),
                                            (5377, (4,)), (6000, (4,)), (7168, (4,)))
             for bpw in bpws for items in (0, 1, 7)]


# Engine 5 (register-stream workers) takes the same blocks up to three per
# worker: the same shapes, plus odd and even landmark counts per item.
_E5_CASES = [(n, bpw, items) for (n, bpw, items) in _E3_CASES if bpw <= 3] + [(5000, 3, 2), (2100, 2, 4)]


@pytest.mark.parametrize("engine,n,bpw,items", [(3,) + c for c in _E3_CASES] + [(5,) + c for c in _E5_CASES])
def test_engine3_tilings(torch, engine, n, bpw, items):
    from gpu_util import TOL32
    L = 23
    s = wl.small_path(n, L, 40 + n % 17, dtype=np.float32)
    rng = np.random.default_rng(n + bpw)
    frames = (s.waypoints[0] + rng.normal(0, 0.02, (2, n, 3))).astype(np.float32)
    lam = landmark_lambda(s.landmarks)
    plan = dict(engine=engine, wg=512, apt=4 * bpw, team=0, aptg=0, batch=0, items=items if items else L)
    _run_exact(torch, s.landmarks, frames, lam, dtype=torch.float32, tol=TOL32,
               name=f"e{engine}_{n}_{bpw}_{items}", plan=plan)


def test_engine3_rejects_structures_it_cannot_hold(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    s = wl.small_path(1800, 3, 5, dtype=np.float32)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), 10.0)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=3, wg=512, apt=4, team=0, aptg=0, batch=0)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=3, wg=512, apt=6, team=0, aptg=0, batch=0)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=3, wg=512, apt=20, team=0, aptg=0, batch=0)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=5, wg=512, apt=4, team=0, aptg=0, batch=0)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=5, wg=512, apt=16, team=0, aptg=0, batch=0)
    cv.close()


def test_engine3_four_blocks_per_wave_default_grid(torch):
    # 7,000 atoms (28 blocks, four per worker, V in FP32 over an item) and
    # 600 landmarks: the default plan with one work item per CU.
    from gpu_util import TOL32
    s = wl.small_path(7000, 600, 77, dtype=np.float32)
    rng = np.random.default_rng(78)
    frames = (s.waypoints[1] + rng.normal(0, 0.02, (2, 7000, 3))).astype(np.float32)
    lam = landmark_lambda(s.landmarks)
    _run_exact(torch, s.landmarks, frames, lam, dtype=torch.float32, tol=TOL32, name="e3_7000x600")


@pytest.mark.parametrize("n,engine,apt", [(2049, 5, 8), (3585, 5, 12), (5376, 5, 12), (5377, 3, 16), (7168, 3, 16),
                                          (7169, 1, None)])
def test_default_plan_by_structure_size(torch, n, engine, apt):
    # Engine 5 takes FP32 structures from 2,049 to 5,376 atoms and engine 3
    # those up to 7,168, each with the fewest blocks per worker that hold
    # them; larger ones go to engine 1.
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    s = wl.small_path(n, 3, 7, dtype=np.float32)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), 10.0)
    assert cv.plan["engine"] == engine
    if apt is not None:
        assert cv.plan["apt"] == apt
    cv.close()


# Multi-landmark engine: structures of one to eight 256-atom blocks
# (K = floor(7 spw / nblk) landmark lanes per step), 23 landmarks (the last
# step is short), fewer landmark lanes than the tiling allows (K = 1 writes a
# single partial per item, K = 2 several), and item counts from one item to
# one landmark per item (items shorter than a step).
_E4_CASES = [(n, spw, K, items) for n in (1, 64, 100, 300, 513, 1000, 1793, 2048) for spw in (2, 3)
             for K, items in ((0, 0), (0, 1), (0, 23), (1, 5), (2, 0))]


@pytest.mark.parametrize("n,spw,K,items", _E4_CASES)
def test_engine4_tilings(torch, n, spw, K, items):
    from gpu_util import TOL32
    L = 23
    s = wl.small_path(n, L, 60 + n % 13, dtype=np.float32)
    rng = np.random.default_rng(n + 7 * spw)
    frames = (s.waypoints[0] + rng.normal(0, 0.02, (2, n, 3))).astype(np.float32)
    lam = landmark_lambda(s.landmarks) if n > 1 else 100.0
    plan = dict(engine=4, wg=512, apt=4 * spw, team=0, aptg=0, batch=K, items=items)
    if K > (7 * spw) // ((n + 63) // 64 * 64 // 256 + ((n + 63) // 64 * 64 % 256 > 0)):
        import paper_1801_02362_amd as pcv
        from gpu_util import dev
        cv = pcv.PathCV(dev(s.landmarks, torch.float32), lam)
        with pytest.raises(pcv.PcvError):
            cv.set_plan(**plan)
        cv.close()
        return
    _run_exact(torch, s.landmarks, frames, lam, dtype=torch.float32, tol=TOL32,
               name=f"e4_{n}_{spw}_{K}_{items}", plan=plan)


def test_engine4_plan_reports_and_rejects(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    # A long landmark set: three units per worker, 21 // 3 = 7 landmark lanes.
    long_set = wl.small_path(700, 1500, 5, dtype=np.float32)
    cv = pcv.PathCV(dev(long_set.landmarks, torch.float32), 10.0)
    p = cv.plan
    assert p["engine"] == 4 and p["apt"] == 12 and p["batch"] == 7
    cv.close()
    # A short one: two units per worker and fewer lanes, so more workgroups share it.
    s = wl.small_path(700, 3, 5, dtype=np.float32)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), 10.0)
    p = cv.plan
    assert p["engine"] == 4 and p["apt"] == 8 and p["batch"] == 1
    cv.set_plan(engine=4, wg=512, apt=8, team=0, aptg=0, batch=0)
    assert cv.plan["batch"] == 4                                      # 14 // 3
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=4, wg=512, apt=8, team=0, aptg=0, batch=5)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=4, wg=512, apt=4, team=0, aptg=0, batch=0)
    cv.close()
    big = wl.small_path(2049, 2, 6, dtype=np.float32)
    cv = pcv.PathCV(dev(big.landmarks, torch.float32), 10.0)
    with pytest.raises(pcv.PcvError):
        cv.set_plan(engine=4, wg=512, apt=12, team=0, aptg=0, batch=0)
    cv.close()


def test_item_counts_and_graph_replay_are_bitwise_stable(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    sysm, frames = wl.path_300x500(50)
    lam = landmark_lambda(sysm.landmarks)
    res = []
    for use_graph in (False, True):
        cv = pcv.PathCV(dev(sysm.landmarks, torch.float32), lam, use_graph=use_graph)
        x = dev(frames[10], torch.float32)
        for _ in range(3):
            o = cv.eval(x)
            res.append(np.concatenate([host(o["sz"]), host(o["ds_dx"]).ravel(), host(o["dz_dx"]).ravel()]))
        cv.close()
    for r in res[1:]:
        assert np.array_equal(r, res[0])


def test_path_lambda_matches_oracle(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    sysm, _ = wl.path_300x500(1)
    cv = pcv.PathCV(dev(sysm.landmarks, torch.float32))
    ref = landmark_lambda(sysm.landmarks)
    assert abs(cv.lam - ref) <= 1e-9 * ref
    cv.close()


def test_nonfinite_input_is_reported(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    sysm, frames = wl.path_22x20(5)
    cv = pcv.PathCV(dev(sysm.landmarks, torch.float64), 500.0)
    x = dev(frames[1], torch.float64)
    x[3, 1] = float("nan")
    o = cv.eval(x)
    assert np.isnan(host(o["sz"])).all()
    with pytest.raises(pcv.PcvError) as ei:
        cv.check()
    assert ei.value.status == -4
    cv.check()   # cleared
    cv.close()


def test_argument_errors(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    sysm, _ = wl.path_22x20(1)
    with pytest.raises(pcv.PcvError) as ei:
        pcv.PathCV(dev(np.zeros((2, 9000, 3)), torch.float32), 1.0)
    assert ei.value.status == -3
    with pytest.raises(pcv.PcvError) as ei:
        pcv.PathCV(dev(sysm.landmarks, torch.float64), -1.0)
    assert ei.value.status == -1
    with pytest.raises(pcv.PcvError):
        pcv.PathCV(dev(sysm.landmarks, torch.float64), 1.0, w=-np.ones(22))


@pytest.mark.parametrize("plan", [None, dict(engine=3, wg=512, apt=4, team=0, aptg=0, batch=0),
                                  dict(engine=5, wg=512, apt=4, team=0, aptg=0, batch=0),
                                  dict(engine=2, wg=512, apt=4, team=16, aptg=2, batch=64),
                                  dict(engine=1, wg=256, apt=1, team=64)])
def test_structure_on_a_landmark(torch, plan):
    """A structure equal to a landmark (D = 0 for it, large lambda): the
    partials' reference property follows the running minimum, so the merge's
    U + (q0 - s) V does not cancel (this case once lost a factor of 20)."""
    from gpu_util import TOL32
    sp = wl.small_path(40, 60, 5, dtype=np.float32)
    lam = landmark_lambda(sp.landmarks)
    frames = np.stack([sp.landmarks[2], sp.landmarks[41]])
    _run_exact(torch, sp.landmarks, frames, lam, dtype=torch.float32, tol=TOL32,
               name=f"on_landmark_{plan['engine'] if plan else 'default'}", plan=plan)


@pytest.mark.parametrize("plan", [dict(engine=1, wg=256, apt=2, team=64),
                                  dict(engine=2, wg=512, apt=4, team=32, aptg=2, batch=13),
                                  dict(engine=3, wg=512, apt=4, team=0, aptg=0, batch=0),
                                  dict(engine=4, wg=512, apt=12, team=0, aptg=0, batch=0),
                                  dict(engine=5, wg=512, apt=4, team=0, aptg=0, batch=0)])
def test_fp32_frame_rounding_is_corrected(torch, plan):
    """A sharp path (lambda ~ 980, 93 atoms, 3,122 landmarks: walker 5 of the
    64-walker batch): s moves by 1.5e-6 when w x_c is rounded to FP32, which
    the FP32 engines 2-5 contract with.  The merges add the first-order term
    dS/dx . (x - x'), so every engine lands within 2e-7 of the oracle; the
    close structure's first (exact) step and the property maps' S_1 = s
    carry the same correction."""
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, check_cv, dev, host, say
    w = wl.walkers(n_walkers=64, n_frames=1)[5]
    lm, f = w.system.landmarks, w.frames[0]
    lam = landmark_lambda(lm)
    ref = path_cv(f.astype(np.float64), lm.astype(np.float64), lam)
    say(f"[rounding] n={lm.shape[1]} L={lm.shape[0]} lam={lam:.1f} plan={plan}")
    cv = pcv.PathCV(dev(lm, torch.float32), lam, use_graph=False)
    cv.set_plan(**plan)
    x = dev(f, torch.float32)
    o = cv.eval(x, grad=True, msd=True)
    sz = host(o["sz"])
    check_cv("exact", TOL32, sz, host(o["ds_dx"]), host(o["dz_dx"]), host(o["msd"]), ref)
    assert abs(sz[0] - ref.s) <= 2e-7, (sz[0], ref.s)
    assert abs(sz[1] - ref.z) <= 2e-7, (sz[1], ref.z)
    c = cv.eval_close(x)
    assert bool(host(c["recomputed"].to(torch.float64))[0])
    assert abs(host(c["sz"])[0] - ref.s) <= 2e-7
    q = torch.arange(1, lm.shape[0] + 1, dtype=torch.float64, device="cuda").reshape(-1, 1)
    p = cv.eval_properties(x, q)
    assert abs(host(p["S"])[0] - ref.s) <= 2e-7
    p2 = cv.eval_properties(x, q, grad=False)
    assert host(p2["S"])[0] == host(p["S"])[0]
    cv.close()


@pytest.mark.parametrize("n,L", [(6000, 8000), (7000, 7000)])
def test_four_blocks_per_wave_at_full_size(torch, n, L):
    """The sizes quoted for engine 3 with four blocks per worker (V kept in
    FP32 over an item, about 31 landmarks per item), path-shaped landmarks
    and a frame between two of them so that the weights spread over
    several landmarks and items: the default plan against the oracle."""
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, check_cv, dev, host, say
    s = wl.small_path(n, L, 90 + n % 7, dtype=np.float32)
    lam = landmark_lambda(s.landmarks)
    rng = np.random.default_rng(n)
    i = L // 3
    f = (0.5 * (s.landmarks[i].astype(np.float64) + s.landmarks[i + 1]) + rng.normal(0, 0.002, (n, 3)))
    f = f.astype(np.float32)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), lam)
    say(f"[exact] four blocks per wave {n} x {L}: plan={cv.plan}")
    assert cv.plan["engine"] == 3 and cv.plan["apt"] == 16
    o = cv.eval(dev(f, torch.float32), msd=True)
    got = host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]), host(o["msd"])
    cv.close()
    ref = path_cv(f.astype(np.float64), s.landmarks.astype(np.float64), lam)
    w = np.exp(-lam * (ref.D - ref.D.min()))
    say(f"[exact] effective landmarks {w.sum() ** 2 / (w ** 2).sum():.1f}, s {ref.s:.4f}")
    check_cv(f"e3_bpw4_{n}x{L}", TOL32, *got, ref)
