"""The allocation-free property-map call (pcv_eval_properties_noalloc)
against pcv_eval_properties, through the C ABI: two calls in a row on one
GPU, the second on a smaller problem (the fixed scratch array keeps the first
call's contents, which the second must not see)."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _case(torch, pcv, sysm, frame, P, seed):
    from gpu_util import dev, host
    rng = np.random.default_rng(seed)
    L, n = sysm.landmarks.shape[0], sysm.landmarks.shape[1]
    Q = rng.normal(size=(L, P))
    Q[:, 0] = np.arange(1, L + 1)
    q = torch.as_tensor(Q, device="cuda")
    x = dev(frame, torch.float32)
    cv = pcv.PathCV(dev(sysm.landmarks, torch.float32), None)
    ref = cv.eval_properties(x, q)
    ref_S, ref_dS = host(ref["S"]).copy(), host(ref["dS_dx"]).copy()
    out = {"S": torch.full((P,), np.nan, dtype=torch.float64, device="cuda"),
           "dS_dx": torch.full((P, n, 3), np.nan, dtype=torch.float32, device="cuda")}
    got = cv.eval_properties_noalloc(x, q, out=out)
    S, dS = host(got["S"]), host(got["dS_dx"])
    cv.check()
    cv.close()
    # The same kernels on the same inputs in the same order: identical results.
    assert np.array_equal(S, ref_S), (S, ref_S)
    assert np.array_equal(dS, ref_dS), np.abs(dS - ref_dS).max()
    assert np.isfinite(S).all() and np.isfinite(dS).all()


def test_noalloc_property_maps_match_the_allocating_call_twice():
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import say
    big, frames = wl.path_300x500(40)
    say("[noalloc] call 1: 300 atoms x 500 landmarks, P = 8")
    _case(torch, pcv, big, frames[30], 8, 3)
    small = wl.small_path(40, 60, 5, dtype=np.float32)
    say("[noalloc] call 2: 40 atoms x 60 landmarks, P = 3")
    _case(torch, pcv, small, small.waypoints[0].astype(np.float32), 3, 4)


def test_noalloc_rejects_scratch_beyond_the_fixed_array():
    import torch
    import paper_1801_02362_amd as pcv
    from gpu_util import dev
    # 300,000 two-atom landmarks with 8 properties: the weights alone need
    # 19.2 MB, beyond the 16 MiB array; rejected before any launch.
    L, P = 300_000, 8
    lm = np.random.default_rng(9).normal(0.0, 0.3, (L, 2, 3)).astype(np.float32)
    cv = pcv.PathCV(dev(lm, torch.float32), 10.0)
    q = torch.zeros(L, P, dtype=torch.float64, device="cuda")
    out = {"S": torch.empty(P, dtype=torch.float64, device="cuda"), "dS_dx": None}
    with pytest.raises(pcv.PcvError) as ei:
        cv.eval_properties_noalloc(dev(lm[0], torch.float32), q, out=out)
    assert ei.value.status == -1
    cv.close()
