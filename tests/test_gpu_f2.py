"""GPU parity of the distance with separate displacement weights w and
alignment weights w' (Section 3.1, Eq. 4 with all its terms) against the FP64
oracle: D_i, s, z and both gradients."""
import numpy as np
import pytest

import workloads as wl
from oracle.path import landmark_lambda, path_cv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _weights(n, seed, zeros=0):
    rng = np.random.default_rng(seed)
    wa = rng.uniform(0.2, 2.0, n)
    wd = rng.uniform(0.0, 3.0, n)
    if zeros:
        wd[rng.choice(n, zeros, replace=False)] = 0.0
    return wa, wd


def _frames(s, n, seed, dtype):
    rng = np.random.default_rng(seed)
    mid = 0.5 * (s.waypoints[0] + s.waypoints[-1])
    base = [s.waypoints[0], mid, s.landmarks[-1]]
    return np.array([(b + rng.normal(0, 0.02, (n, 3))) for b in base]).astype(dtype)


def _run(torch, n, L, seed, dtype, tol, name, zeros=0, use_graph=True):
    import paper_1801_02362_amd as pcv
    from gpu_util import check_cv, dev, host, say
    np_dt = np.float32 if dtype == torch.float32 else np.float64
    s = wl.small_path(n, L, seed, dtype=np_dt)
    wa, wd = _weights(n, seed + 1, zeros)
    lam = landmark_lambda(s.landmarks, w=wd, wp=wa) if n > 1 else 100.0
    frames = _frames(s, n, seed + 2, np_dt)
    say(f"[f2] {name}: n={n} L={L} frames={len(frames)} graph={use_graph}")
    cv = pcv.PathCV(dev(s.landmarks, dtype), lam, w=wa, use_graph=use_graph)
    cv.set_displacement_weights(wd)
    x = torch.empty(n, 3, dtype=dtype, device="cuda")
    for rep in range(2):                       # the second pass replays the graph
        for t, f in enumerate(frames):
            x.copy_(torch.as_tensor(f))
            o = cv.eval(x, grad=True, msd=True)
            ref = path_cv(f.astype(np.float64), s.landmarks.astype(np.float64), lam, w=wd, wp=wa)
            check_cv(f"{name}[{rep}.{t}]", tol, host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"]),
                     host(o["msd"]), ref)
    cv.check()
    st = cv.stats()
    assert st["exact_evals"] == 2 * len(frames)
    assert st["expensive_msd"] == 2 * len(frames) * L
    cv.close()


@pytest.mark.parametrize("n,L,seed", [(150, 60, 3), (97, 37, 5), (1, 4, 6), (700, 300, 7), (2049, 23, 8)])
def test_fp32(torch, n, L, seed):
    from gpu_util import TOL32
    _run(torch, n, L, seed, torch.float32, TOL32, f"fp32_{n}x{L}", zeros=n // 10)


@pytest.mark.parametrize("n,L,seed", [(22, 20, 11), (130, 45, 12)])
def test_fp64(torch, n, L, seed):
    from gpu_util import TOL64
    _run(torch, n, L, seed, torch.float64, TOL64, f"fp64_{n}x{L}", zeros=3)


def test_without_graphs(torch):
    from gpu_util import TOL32
    _run(torch, 64, 33, 21, torch.float32, TOL32, "nograph", use_graph=False)


def test_equal_weights_match_the_engine_path(torch):
    """w = w': the three-pass path and the engines give the same CV."""
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    s = wl.small_path(120, 50, 31, dtype=np.float32)
    wa, _ = _weights(120, 32)
    lam = landmark_lambda(s.landmarks, w=wa)
    x = dev(_frames(s, 120, 33, np.float32)[1], torch.float32)
    a = pcv.PathCV(dev(s.landmarks, torch.float32), lam, w=wa)
    b = pcv.PathCV(dev(s.landmarks, torch.float32), lam, w=wa)
    b.set_displacement_weights(3.0 * wa)            # normalised: the same weights
    oa, ob = a.eval(x, msd=True), b.eval(x, msd=True)
    # each side within its own bound of the exact values: twice the bound apart
    assert np.allclose(host(oa["sz"]), host(ob["sz"]), atol=2e-6, rtol=0)
    assert np.allclose(host(oa["msd"]), host(ob["msd"]), rtol=2e-5, atol=1e-12)
    for k in ("ds_dx", "dz_dx"):
        ga, gb = host(oa[k]), host(ob[k])
        assert np.abs(ga - gb).max() <= 2e-5 * np.abs(ga).max()
    b.set_displacement_weights(None)                # off again: the engine path
    oc = b.eval(x, msd=True)
    assert np.allclose(host(oa["sz"]), host(oc["sz"]), atol=1e-9, rtol=0)
    a.close()
    b.close()


def test_modes_it_does_not_combine_with(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    s = wl.small_path(30, 12, 41, dtype=np.float32)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), 40.0)
    x = dev(s.landmarks[3], torch.float32)
    with pytest.raises(ValueError):
        cv.set_displacement_weights(np.ones(29))
    for bad in (-np.ones(30), np.zeros(30), np.full(30, np.nan)):
        with pytest.raises(pcv.PcvError):
            cv.set_displacement_weights(bad)
    cv.set_displacement_weights(np.linspace(0.0, 1.0, 30))
    with pytest.raises(pcv.PcvError):
        cv.eval_close(x)
    with pytest.raises(pcv.PcvError):
        cv.update_close(x)
    with pytest.raises(pcv.PcvError):
        cv.set_neighbour_list(4, 2)
    q = torch.ones(12, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(pcv.PcvError):
        cv.eval_properties(x, q)
    cv.eval(x)
    cv.set_displacement_weights(None)
    cv.set_neighbour_list(4, 2)
    with pytest.raises(pcv.PcvError):
        cv.set_displacement_weights(np.ones(30))
    cv.set_neighbour_list(0, 1)
    cv.set_displacement_weights(np.ones(30))
    cv.eval(x)
    cv.check()
    cv.close()


def test_nonfinite_input_is_reported(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    s = wl.small_path(40, 10, 51, dtype=np.float32)
    cv = pcv.PathCV(dev(s.landmarks, torch.float32), 40.0)
    cv.set_displacement_weights(np.arange(1, 41, dtype=np.float64))
    bad = s.landmarks[2].copy()
    bad[7, 1] = np.inf
    cv.eval(dev(bad, torch.float32))
    with pytest.raises(pcv.PcvError):
        cv.check()
    cv.eval(dev(s.landmarks[2], torch.float32))
    cv.check()
    cv.close()
