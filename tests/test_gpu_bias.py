"""GPU parity of the metadynamics bias (Eq. 1 on (s, z), grid with bicubic
Hermite interpolation, atom gradient) against the FP64 oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import bias as ob
from oracle.path import landmark_lambda, path_cv

pytestmark = pytest.mark.gpu

_GRID = dict(s_min=0.5, s_max=6.5, ns=41, z_min=-0.2, z_max=0.4, nz=31, height=1.3, sigma_s=0.4, sigma_z=0.05)
_HILLS = [(2.0, 0.1), (4.4, -0.05), (3.3, 0.3), (3.31, 0.29), (6.4, 0.39)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _pair(torch, grid=_GRID, hills=_HILLS):
    import paper_1801_02362_amd as pcv
    g = grid
    b = pcv.Bias((g["s_min"], g["s_max"]), (g["z_min"], g["z_max"]), (g["ns"], g["nz"]), g["height"],
                 (g["sigma_s"], g["sigma_z"]))
    og = ob.Grid(**g)
    for s0, z0 in hills:
        b.deposit(torch.tensor([s0, z0], dtype=torch.float64, device="cuda"))
        ob.deposit(og, s0, z0)
    return b, og


def test_grid_matches_oracle_after_deposits(torch):
    from gpu_util import say
    say("[bias] grid after 5 deposits, 41 x 31 nodes")
    b, og = _pair(torch)
    got = b.grid()
    assert b.hills() == len(_HILLS)
    for c in range(4):
        scale = np.abs(og.data[c]).max()
        assert np.abs(got[c] - og.data[c]).max() <= 1e-13 * scale, c
    b.close()


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_gradient_matches_oracle_inside_on_nodes_and_outside(torch, dtype_name):
    from gpu_util import say
    dtype = getattr(torch, dtype_name)
    say(f"[bias] interpolation and atom gradient, {dtype_name}")
    b, og = _pair(torch)
    rng = np.random.default_rng(5)
    n = 37
    ds = rng.normal(size=(n, 3)).astype(np.float32 if dtype_name == "float32" else np.float64)
    dz = rng.normal(size=(n, 3)).astype(ds.dtype)
    pts = list(zip(rng.uniform(0.5, 6.5, 12), rng.uniform(-0.2, 0.4, 12)))
    pts += [(0.5, -0.2), (6.5, 0.4), (0.5 + 7 * og.hs, -0.2 + 4 * og.hz), (3.3, 0.3), (2.0000001, 0.1)]
    pts += [(0.49, 0.0), (6.51, 0.0), (3.0, -0.21), (3.0, 0.41)]
    dsd, dzd = torch.as_tensor(ds, device="cuda"), torch.as_tensor(dz, device="cuda")
    for s, z in pts:
        grad, v, ok = b.gradient(torch.tensor([s, z], dtype=torch.float64, device="cuda"), dsd, dzd)
        V, Vs, Vz, rok, rg = ob.bias_gradient(og, s, z, ds, dz)
        v = v.cpu().numpy()
        assert int(ok.item()) == int(rok), (s, z)
        scale = og.height * 40.0
        assert abs(v[0] - V) <= 1e-12 * og.height, (s, z)
        assert abs(v[1] - Vs) <= 1e-12 * scale and abs(v[2] - Vz) <= 1e-12 * scale / 0.05, (s, z)
        g = grad.double().cpu().numpy()
        tol = (1e-12 if dtype_name == "float64" else 1e-6) * max(1e-30, np.abs(rg).max())
        assert np.abs(g - rg).max() <= tol, (s, z)
    b.close()


def test_nonfinite_cv_values_deposit_nothing(torch):
    b, og = _pair(torch, hills=[(3.0, 0.1)])
    before = b.grid()
    b.deposit(torch.tensor([float("nan"), 0.1], dtype=torch.float64, device="cuda"))
    b.deposit(torch.tensor([3.0, float("inf")], dtype=torch.float64, device="cuda"))
    assert np.array_equal(b.grid(), before)
    b.close()


def test_large_structure_gradient(torch):
    from gpu_util import say
    say("[bias] gradient on 5000 atoms (multi-workgroup)")
    b, og = _pair(torch)
    rng = np.random.default_rng(8)
    ds = rng.normal(size=(5000, 3)).astype(np.float32)
    dz = rng.normal(size=(5000, 3)).astype(np.float32)
    s, z = 3.21, 0.17
    grad, v, ok = b.gradient(torch.tensor([s, z], dtype=torch.float64, device="cuda"),
                             torch.as_tensor(ds, device="cuda"), torch.as_tensor(dz, device="cuda"))
    _, _, _, _, rg = ob.bias_gradient(og, s, z, ds, dz)
    assert np.abs(grad.double().cpu().numpy() - rg).max() <= 1e-6 * np.abs(rg).max()
    b.close()


def test_bias_on_the_path_variables_end_to_end(torch):
    """Exact path CV (FP32) -> bias gradient on the device, against the oracle
    CVs and the oracle bias gradient."""
    import paper_1801_02362_amd as pcv
    from gpu_util import say
    say("[bias] path CV + bias, 40 atoms x 30 landmarks")
    sp = wl.small_path(40, 30, 31, dtype=np.float32)
    lam = landmark_lambda(sp.landmarks)
    x = (sp.waypoints[1] + np.random.default_rng(9).normal(0, 0.02, (40, 3))).astype(np.float32)
    ref = path_cv(x.astype(np.float64), sp.landmarks.astype(np.float64), lam)
    grid = dict(s_min=ref.s - 4, s_max=ref.s + 4, ns=81, z_min=ref.z - 0.2, z_max=ref.z + 0.2, nz=81,
                height=2.0, sigma_s=0.6, sigma_z=0.04)
    hills = [(ref.s - 0.5, ref.z + 0.02), (ref.s + 0.2, ref.z - 0.01), (ref.s, ref.z)]
    b, og = _pair(torch, grid, hills)
    cv = pcv.PathCV(torch.as_tensor(sp.landmarks, device="cuda"), lam)
    o = cv.eval(torch.as_tensor(x, device="cuda"))
    grad, v, ok = b.gradient(o["sz"], o["ds_dx"], o["dz_dx"])
    V, Vs, Vz, rok, rg = ob.bias_gradient(og, ref.s, ref.z, ref.ds_dx, ref.dz_dx)
    v = v.cpu().numpy()
    assert int(ok.item()) == 1 and rok
    # the CVs agree to 1e-6 (s, z) and 1e-5 (gradients) relative; the bias follows
    assert abs(v[0] - V) <= 1e-5 * abs(V) + 1e-9
    assert np.abs(grad.double().cpu().numpy() - rg).max() <= 1e-4 * np.abs(rg).max()
    cv.close()
    b.close()
