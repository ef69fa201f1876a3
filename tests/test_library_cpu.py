"""CPU checks of the native library: it loads, exports every entry point that
include/pcv.h declares, and the per-landmark FP64 math (host build of the
same header the kernels inline) agrees with the oracle."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import workloads as wl
from oracle.msd import quaternion_matrix, rotation_adjoint, superpose

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1801_02362_amd")


def _declared():
    txt = open(os.path.join(ROOT, "include", "pcv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pcv_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_entry_point():
    lib = ctypes.CDLL(os.path.join(PKG, "libpcv.so"))
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_loads_library():
    import paper_1801_02362_amd as pcv
    L = pcv.load_library()
    assert L.pcv_max_atoms(32) >= 5000
    assert L.pcv_status_string(-4) == b"non-finite input"


@pytest.fixture(scope="module")
def hm():
    L = ctypes.CDLL(os.path.join(PKG, "libpcv_hosttest.so"))
    P = ctypes.POINTER(ctypes.c_double)
    L.pcvt_superpose.argtypes = [P, ctypes.c_double, P, P, P, P]
    L.pcvt_superpose.restype = ctypes.c_int
    L.pcvt_char_poly.argtypes = [P, P]
    L.pcvt_jacobi_top.argtypes = [P, P]
    L.pcvt_jacobi_top.restype = ctypes.c_double
    L.pcvt_rotation_adjoint.argtypes = [P, ctypes.c_double, P, P, P]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _native(hm, M, lam_up):
    M = np.ascontiguousarray(M, dtype=np.float64)
    lam = np.zeros(1); q = np.zeros(4); R = np.zeros(9); F = np.zeros(10)
    fb = hm.pcvt_superpose(_p(M), lam_up, _p(lam), _p(q), _p(R), _p(F))
    return fb, lam[0], q, R.reshape(3, 3), F


@pytest.mark.parametrize("seed", range(8))
def test_native_superposition_matches_oracle(hm, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 40))
    x = rng.normal(0, 0.3, (n, 3))
    a, _, _ = wl.rigid_copy(x + rng.normal(0, 0.1 * (seed % 4 + 1), (n, 3)), seed)
    sp = superpose(x, a)
    w = np.full(n, 1 / n)
    Gx, Ga = np.sum(w[:, None] * sp.x_c ** 2), np.sum(w[:, None] * sp.a_c ** 2)
    fb, lam, q, R, _ = _native(hm, sp.M, 0.5 * (Gx + Ga))
    assert fb == 0
    assert abs(lam - sp.evals[0]) <= 2e-16 * (Gx + Ga) * 8
    assert abs((Gx + Ga - 2 * lam) - float(sp.D)) < 1e-15
    assert np.abs(R - sp.R).max() < 1e-12


def test_char_poly_matches_numpy(hm):
    rng = np.random.default_rng(3)
    for _ in range(5):
        M = np.ascontiguousarray(rng.normal(size=(3, 3)))
        c = np.zeros(3)
        hm.pcvt_char_poly(_p(M), _p(c))
        ref = np.poly(quaternion_matrix(M))
        assert abs(ref[1]) < 1e-12
        assert np.allclose(c, ref[2:], rtol=1e-12, atol=1e-12)


def test_degenerate_spectrum_uses_jacobi(hm):
    # Collinear atoms: rotation about the line is free, the top eigenvalue is double.
    x = np.outer(np.linspace(-1, 1, 6), [0.3, -0.2, 0.5])
    a, _, _ = wl.rigid_copy(x, 4)
    sp = superpose(x, a)
    w = np.full(6, 1 / 6)
    Gx, Ga = np.sum(w[:, None] * sp.x_c ** 2), np.sum(w[:, None] * sp.a_c ** 2)
    fb, lam, q, R, _ = _native(hm, sp.M, 0.5 * (Gx + Ga))
    assert fb == 1
    assert abs((Gx + Ga - 2 * lam) - float(sp.D)) < 1e-14
    assert abs(np.linalg.det(R) - 1) < 1e-12
    # R still superposes the line: residual distance equals the optimum.
    d = sp.x_c - sp.a_c @ R.T
    assert abs(np.sum(w[:, None] * d * d) - float(sp.D)) < 1e-14


def test_zero_correlation(hm):
    fb, lam, q, R, _ = _native(hm, np.zeros((3, 3)), 0.0)
    assert lam == 0.0 and abs(np.linalg.det(R) - 1) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_native_rotation_adjoint_matches_oracle(hm, seed):
    rng = np.random.default_rng(10 + seed)
    n = 12
    x = rng.normal(0, 0.3, (n, 3))
    y, _, _ = wl.rigid_copy(x + rng.normal(0, 0.05, (n, 3)), seed)
    sp = superpose(x, y)
    w = np.full(n, 1 / n)
    Gx, Ga = np.sum(w[:, None] * sp.x_c ** 2), np.sum(w[:, None] * sp.a_c ** 2)
    fb, lam, q, R, F = _native(hm, sp.M, 0.5 * (Gx + Ga))
    G = np.ascontiguousarray(rng.normal(size=(3, 3)))
    Gam = np.zeros(9)
    hm.pcvt_rotation_adjoint(_p(F), lam, _p(np.ascontiguousarray(q)), _p(G), _p(Gam))
    ref = rotation_adjoint(sp.evals, sp.evecs, G)
    assert np.abs(Gam.reshape(3, 3) - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_header_compiles_as_c(tmp_path):
    """include/pcv.h is a C header: a C99 translation unit that includes it
    and calls into it compiles with warnings as errors."""
    src = tmp_path / "t.c"
    src.write_text('#include "pcv.h"\nint main(void) { pcv_options o; pcv_default_options(&o); return o.device; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", f"-I{os.path.join(ROOT, 'include')}",
                        "-c", str(src), "-o", str(tmp_path / "t.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_host_math_under_address_and_undefined_sanitizers(tmp_path):
    """The superposition math the kernels inline (pcv_math.h, through
    pcv_hosttest.cpp), built for the host with AddressSanitizer and
    UndefinedBehaviorSanitizer and run over random and degenerate inputs."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "host_sanitize"
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined", "-fno-sanitize-recover=all", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{os.path.join(PKG, 'csrc')}", os.path.join(ROOT, "tests", "host_sanitize_main.cpp"),
           os.path.join(PKG, "csrc", "pcv_hosttest.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-2000:]
    assert "0 non-finite" in r.stdout
