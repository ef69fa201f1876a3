"""Path collective variables with a floating close structure on MI355X.

Thin Python binding over the C ABI in ``include/pcv.h`` (``libpcv.so``, built
by ``python -m paper_1801_02362_amd.build``).  This module only marshals
arguments: every step of the computation runs in the HIP kernels.  PyTorch
supplies device memory and the stream; tensors must live on the GPU.

Method: Pazurikova et al., arXiv:1801.02362 -- Eq. 2 (property-map / path
CV), Eq. 3-4 (exact MSD and derivative), Algorithm 2 with Eq. 5-6 (floating
close structure).
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["PcvError", "PathCV", "BatchPathCV", "Surrogate", "Bias", "library_path", "load_library", "FP32", "FP64"]

_HERE = os.path.dirname(os.path.abspath(__file__))
FP32, FP64 = 32, 64
_STATUS = {0: "ok", -1: "invalid argument", -2: "invalid call order", -3: "unsupported size",
           -4: "non-finite input", -5: "HIP runtime error", -6: "out of device memory",
           -7: "unsupported"}


class PcvError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        self.status = status
        super().__init__(f"pcv status {status} ({_STATUS.get(status, '?')}): {message}")


class _Options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("precision", ctypes.c_int),
                ("eps", ctypes.c_double), ("use_graph", ctypes.c_int)]


class _BiasOptions(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("s_min", ctypes.c_double),
                ("s_max", ctypes.c_double), ("ns", ctypes.c_int), ("z_min", ctypes.c_double),
                ("z_max", ctypes.c_double), ("nz", ctypes.c_int), ("height", ctypes.c_double),
                ("sigma_s", ctypes.c_double), ("sigma_z", ctypes.c_double)]


class _Plan(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("engine", "wg", "apt", "team", "aptg", "batch", "grid", "items")]


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("frames", "recomputes", "expensive_msd", "approx_frames", "exact_evals", "eigen_fallbacks")]


class _MlpStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("surrogate_steps", ctypes.c_int64), ("exact_steps", ctypes.c_int64),
                ("judged_steps", ctypes.c_int64), ("max_abs_ds", ctypes.c_double), ("max_abs_dz", ctypes.c_double),
                ("mean_abs_ds", ctypes.c_double), ("mean_abs_dz", ctypes.c_double)]


_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "libpcv.so")


def load_library():
    """Load ``libpcv.so`` from the package directory; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1801_02362_amd.build`")
    L = ctypes.CDLL(path)
    vp, i, d, st = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int
    sig = {
        "pcv_default_options": (None, [ctypes.POINTER(_Options)]),
        "pcv_create": (st, [ctypes.POINTER(vp), ctypes.POINTER(_Options)]),
        "pcv_destroy": (st, [vp]),
        "pcv_load_landmarks": (st, [vp, i, i, vp, vp, vp, d]),
        "pcv_max_atoms": (i, [i]),
        "pcv_path_lambda": (st, [vp, d, ctypes.POINTER(d)]),
        "pcv_set_lambda": (st, [vp, d]),
        "pcv_eval": (st, [vp, vp, vp, vp, vp, vp]),
        "pcv_eval_close": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "pcv_force_reassign": (st, [vp]),
        "pcv_update_close": (st, [vp, vp]),
        "pcv_get_stats": (st, [vp, ctypes.POINTER(_Stats)]),
        "pcv_reset_stats": (st, [vp]),
        "pcv_check": (st, [vp]),
        "pcv_get_plan": (st, [vp, ctypes.POINTER(_Plan)]),
        "pcv_set_plan": (st, [vp, ctypes.POINTER(_Plan)]),
        "pcv_set_kernel_timing": (st, [vp, i]),
        "pcv_get_kernel_timing": (st, [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64)]),
        "pcv_status_string": (ctypes.c_char_p, [st]),
        "pcv_last_error": (ctypes.c_char_p, [vp]),
        "pcv_batch_create": (st, [ctypes.POINTER(vp), ctypes.POINTER(_Options)]),
        "pcv_batch_destroy": (st, [vp]),
        "pcv_batch_load": (st, [vp, i, vp, vp, vp, vp]),
        "pcv_batch_plan": (st, [vp, i, ctypes.c_char_p]),
        "pcv_batch_eval": (st, [vp, vp, vp, vp, vp]),
        "pcv_batch_plan_string": (ctypes.c_char_p, [vp]),
        "pcv_batch_set_kernel_timing": (st, [vp, i]),
        "pcv_batch_get_kernel_timing": (st, [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64)]),
        "pcv_batch_last_error": (ctypes.c_char_p, [vp]),
        "pcv_mlp_create": (st, [ctypes.POINTER(vp), ctypes.POINTER(_Options), i, i, i, vp, vp]),
        "pcv_mlp_destroy": (st, [vp]),
        "pcv_mlp_param_count": (ctypes.c_longlong, [vp]),
        "pcv_mlp_set_params": (st, [vp, vp, ctypes.c_longlong]),
        "pcv_mlp_get_params": (st, [vp, vp, ctypes.c_longlong]),
        "pcv_mlp_get_grads": (st, [vp, vp, ctypes.c_longlong]),
        "pcv_mlp_set_scaling": (st, [vp, vp, vp]),
        "pcv_mlp_align": (st, [vp, vp, i, vp, vp]),
        "pcv_mlp_forward": (st, [vp, vp, i, vp]),
        "pcv_mlp_train_step": (st, [vp, vp, vp, i, ctypes.c_float, vp]),
        "pcv_mlp_eval": (st, [vp, vp, i, vp, vp, vp]),
        "pcv_mlp_step": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "pcv_mlp_get_stats": (st, [vp, ctypes.POINTER(_MlpStats)]),
        "pcv_mlp_reset_stats": (st, [vp]),
        "pcv_mlp_save_state": (st, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
        "pcv_mlp_load_state": (st, [vp, vp, ctypes.c_size_t]),
        "pcv_mlp_last_error": (ctypes.c_char_p, [vp]),
        "pcv_set_neighbour_list": (st, [vp, i, i]),
        "pcv_eval_properties": (st, [vp, vp, i, vp, vp, vp]),
        "pcv_eval_properties_noalloc": (st, [vp, vp, i, vp, vp, vp]),
        "pcv_stream_read": (st, [vp, ctypes.c_size_t, vp, i, vp]),
        "pcv_set_displacement_weights": (st, [vp, vp]),
        "pcv_save_state": (st, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
        "pcv_load_state": (st, [vp, vp, ctypes.c_size_t]),
        "pcv_get_neighbour_list": (st, [vp, vp, i, ctypes.POINTER(i)]),
        "pcv_bias_create": (st, [ctypes.POINTER(vp), ctypes.POINTER(_BiasOptions)]),
        "pcv_bias_destroy": (st, [vp]),
        "pcv_bias_deposit": (st, [vp, vp]),
        "pcv_bias_gradient": (st, [vp, vp, i, i, vp, vp, vp, vp, vp]),
        "pcv_bias_hills": (st, [vp, ctypes.POINTER(ctypes.c_longlong)]),
        "pcv_bias_get_grid": (st, [vp, vp]),
        "pcv_bias_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _as_host_f64(a, size, what):
    if a is None:
        return None, None
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if arr.size != size:
        raise ValueError(f"{what} must have {size} entries")
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


class PathCV:
    """Path CVs of one structure against a landmark set on one GPU.

    ``landmarks``: CUDA tensor ``[L][n][3]`` (float32 -> FP32 path, float64 ->
    FP64 path).  ``lam``: sharpness; if None it is set to
    ``lambda_factor / mean D(a_i, a_{i+1})`` computed on the device.
    ``q``: per-landmark property (default 1..L).  ``w``: per-atom weights.
    ``eps``: close-structure threshold (nm^2).
    """

    def __init__(self, landmarks, lam: float | None = None, *, q=None, w=None, eps: float = 0.01,
                 lambda_factor: float = 2.3, use_graph: bool = False, stream=None, device: int | None = None):
        import torch
        L = load_library()
        if not (landmarks.is_cuda and landmarks.dim() == 3 and landmarks.shape[2] == 3):
            raise ValueError("landmarks must be a CUDA tensor [L][n][3]")
        if landmarks.dtype not in (torch.float32, torch.float64):
            raise ValueError("landmarks must be float32 or float64")
        self._L = L
        self.dtype = landmarks.dtype
        self.n_landmarks, self.n_atoms = int(landmarks.shape[0]), int(landmarks.shape[1])
        self.device = landmarks.device if device is None else torch.device("cuda", device)
        self._stream = stream
        opt = _Options()
        L.pcv_default_options(ctypes.byref(opt))
        opt.device = self.device.index if self.device.index is not None else torch.cuda.current_device()
        opt.stream = _stream_ptr(stream).value
        opt.precision = FP64 if self.dtype == torch.float64 else FP32
        opt.eps = float(eps)
        opt.use_graph = 1 if use_graph else 0
        h = ctypes.c_void_p()
        self._check(L.pcv_create(ctypes.byref(h), ctypes.byref(opt)), None)
        self._h = h
        lm = landmarks.contiguous()
        qa, qp = _as_host_f64(q, self.n_landmarks, "q")   # qa, wa keep the buffers alive for the call
        self._q_keep = q
        wa, wp = _as_host_f64(w, self.n_atoms, "w")
        self._check(L.pcv_load_landmarks(h, self.n_atoms, self.n_landmarks, _ptr(lm), qp, wp,
                                         ctypes.c_double(1.0 if lam is None else float(lam))))
        del qa, wa
        if lam is None:
            out = ctypes.c_double()
            self._check(L.pcv_path_lambda(h, ctypes.c_double(lambda_factor), ctypes.byref(out)))
            lam = out.value
            self._check(L.pcv_set_lambda(h, ctypes.c_double(lam)))
        self.lam = float(lam)
        self._out = {}

    # -- helpers --------------------------------------------------------
    def _check(self, status, h="self"):
        if status != 0:
            msg = ""
            if h == "self" and getattr(self, "_h", None) is not None:
                msg = (self._L.pcv_last_error(self._h) or b"").decode()
            raise PcvError(status, msg)

    def _outputs(self, grad, with_msd, close):
        import torch
        key = (grad, with_msd, close)
        if key not in self._out:
            dev = self.device
            o = {"sz": torch.empty(2, dtype=torch.float64, device=dev)}
            if grad:
                o["ds_dx"] = torch.empty(self.n_atoms, 3, dtype=self.dtype, device=dev)
                o["dz_dx"] = torch.empty(self.n_atoms, 3, dtype=self.dtype, device=dev)
            if with_msd:
                o["msd"] = torch.empty(self.n_landmarks, dtype=torch.float64, device=dev)
            if close:
                o["recomputed"] = torch.empty(1, dtype=torch.int32, device=dev)
            self._out[key] = o
        return self._out[key]

    def _check_x(self, x):
        if not (x.is_cuda and x.dtype == self.dtype and tuple(x.shape) == (self.n_atoms, 3) and x.is_contiguous()):
            raise ValueError(f"x must be a contiguous CUDA {self.dtype} tensor of shape ({self.n_atoms}, 3)")

    # -- Algorithm 1 ----------------------------------------------------
    def eval(self, x, *, grad: bool = True, msd: bool = False, out: dict | None = None) -> dict:
        """Exact s, z (``out['sz']``), gradients and optionally every D_i.
        Results are written asynchronously on the handle's stream; the
        returned tensors are reused by later calls unless ``out`` is given."""
        self._check_x(x)
        o = out if out is not None else self._outputs(grad, msd, False)
        self._check(self._L.pcv_eval(self._h, _ptr(x), _ptr(o["sz"]), _ptr(o.get("ds_dx")),
                                     _ptr(o.get("dz_dx")), _ptr(o.get("msd"))))
        return o

    # -- Algorithm 2 ----------------------------------------------------
    def eval_close(self, x, *, grad: bool = True, msd: bool = False, out: dict | None = None) -> dict:
        """One close-structure step; ``out['recomputed']`` is 1 on a
        reassignment step, 0 on an approximate step."""
        self._check_x(x)
        o = out if out is not None else self._outputs(grad, msd, True)
        self._check(self._L.pcv_eval_close(self._h, _ptr(x), _ptr(o["sz"]), _ptr(o.get("ds_dx")),
                                           _ptr(o.get("dz_dx")), _ptr(o.get("msd")),
                                           _ptr(o.get("recomputed"))))
        return o

    def update_close(self, x):
        self._check_x(x)
        self._check(self._L.pcv_update_close(self._h, _ptr(x)))

    def force_reassign(self):
        self._check(self._L.pcv_force_reassign(self._h))

    def eval_properties(self, x, q, *, grad: bool = True, out: dict | None = None) -> dict:
        """Property-map components S [P] and gradients [P][n][3] for the
        device properties ``q`` (float64 [L][P], P <= 8); see
        ``pcv_eval_properties``."""
        import torch
        self._check_x(x)
        if not (q.is_cuda and q.dtype == torch.float64 and q.dim() == 2 and q.shape[0] == self.n_landmarks
                and q.is_contiguous()):
            raise ValueError("q must be a contiguous CUDA float64 tensor [L][P]")
        P = int(q.shape[1])
        o = out or {}
        S = o.get("S") if o.get("S") is not None else torch.empty(P, dtype=torch.float64, device=x.device)
        dS = None
        if grad:
            dS = o.get("dS_dx") if o.get("dS_dx") is not None else torch.empty(P, x.shape[0], 3, dtype=x.dtype,
                                                                                device=x.device)
        self._check(self._L.pcv_eval_properties(self._h, _ptr(x), P, _ptr(q), _ptr(S), _ptr(dS)))
        return {"S": S, "dS_dx": dS}

    def eval_properties_noalloc(self, x, q, *, out: dict) -> dict:
        """As ``eval_properties`` with caller-provided outputs (``out["S"]``
        [P] float64 and ``out["dS_dx"]`` [P][n][3] or None) and the library's
        fixed device scratch: the call allocates nothing
        (``pcv_eval_properties_noalloc``)."""
        import torch
        self._check_x(x)
        if not (q.is_cuda and q.dtype == torch.float64 and q.dim() == 2 and q.shape[0] == self.n_landmarks
                and q.is_contiguous()):
            raise ValueError("q must be a contiguous CUDA float64 tensor [L][P]")
        P = int(q.shape[1])
        S, dS = out["S"], out.get("dS_dx")
        if not (S.is_cuda and S.dtype == torch.float64 and S.numel() == P and S.is_contiguous()):
            raise ValueError("out['S'] must be a contiguous CUDA float64 tensor [P]")
        if dS is not None and not (dS.is_cuda and dS.dtype == x.dtype and tuple(dS.shape) == (P, x.shape[0], 3)
                                   and dS.is_contiguous()):
            raise ValueError("out['dS_dx'] must be a contiguous CUDA tensor [P][n][3] of the coordinate type")
        self._check(self._L.pcv_eval_properties_noalloc(self._h, _ptr(x), P, _ptr(q), _ptr(S), _ptr(dS)))
        return {"S": S, "dS_dx": dS}

    def set_displacement_weights(self, w_disp=None):
        """Per-atom displacement weights ``w`` of the distance, separate from
        the alignment weights given at construction (``None``: off).  See
        ``pcv_set_displacement_weights``."""
        arr, wp = _as_host_f64(w_disp, self.n_atoms, "w_disp")
        self._check(self._L.pcv_set_displacement_weights(self._h, wp))
        del arr

    def save_state(self) -> bytes:
        """Checkpoint of the close structure, counters and neighbour list
        (``pcv_save_state``)."""
        n = ctypes.c_size_t(0)
        self._check(self._L.pcv_save_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._L.pcv_save_state(self._h, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)))
        return buf.raw[:n.value]

    def load_state(self, state: bytes):
        """Resume from ``save_state`` output (``pcv_load_state``)."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        self._check(self._L.pcv_load_state(self._h, ctypes.cast(buf, ctypes.c_void_p), len(state)))

    def set_neighbour_list(self, M: int, stride: int = 1):
        """Neighbour list of the ``M`` nearest references refreshed every
        ``stride`` calls (``M = 0``: off).  See ``pcv_set_neighbour_list``."""
        self._check(self._L.pcv_set_neighbour_list(self._h, int(M), int(stride)))

    def neighbour_list(self):
        """Current members (host int array, empty when off)."""
        import numpy as np
        cnt = ctypes.c_int()
        self._check(self._L.pcv_get_neighbour_list(self._h, None, 0, ctypes.byref(cnt)))
        out = np.empty(cnt.value, dtype=np.int32)
        if cnt.value:
            self._check(self._L.pcv_get_neighbour_list(self._h, out.ctypes.data_as(ctypes.c_void_p), cnt.value,
                                                        ctypes.byref(cnt)))
        return out

    def stats(self) -> dict:
        st = _Stats()
        self._check(self._L.pcv_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def reset_stats(self):
        self._check(self._L.pcv_reset_stats(self._h))

    def check(self):
        """Synchronise and raise PcvError(-4) if a non-finite input was seen."""
        self._check(self._L.pcv_check(self._h))

    @property
    def plan(self) -> dict:
        """Tiling of the landmark streaming kernel (see ``pcv_plan`` in pcv.h)."""
        p = _Plan()
        self._check(self._L.pcv_get_plan(self._h, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in _Plan._fields_}

    def set_plan(self, engine: int = 1, wg: int = 256, apt: int = 1, team: int = 16, aptg: int = 0,
                 batch: int = 1, items: int = 0):
        p = _Plan(engine, wg, apt, team, aptg, batch, 0, items)
        self._check(self._L.pcv_set_plan(self._h, ctypes.byref(p)))

    def set_kernel_timing(self, enable: bool):
        """Record HIP events around every landmark-kernel launch (calls run
        eagerly while enabled)."""
        self._check(self._L.pcv_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_timing(self) -> tuple[float, int]:
        """(summed landmark-kernel milliseconds, launches) since enabling."""
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        self._check(self._L.pcv_get_kernel_timing(self._h, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._L.pcv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPathCV:
    """Many independent walkers (structure + landmark set each, uneven sizes)
    evaluated exactly by one persistent engine launch.

    ``landmarks``: list of CUDA tensors ``[L_w][n_w][3]`` (same dtype);
    ``lams``: one sharpness per walker.
    """

    def __init__(self, landmarks, lams, *, use_graph: bool = True, tune: bool = False,
                 cache_path: str | None = None, stream=None):
        import torch
        L = load_library()
        self._L = L
        self.dtype = landmarks[0].dtype
        self.device = landmarks[0].device
        self.n = [int(t.shape[1]) for t in landmarks]
        self.Ls = [int(t.shape[0]) for t in landmarks]
        self.W = len(landmarks)
        self.atom_off = [0]
        for v in self.n:
            self.atom_off.append(self.atom_off[-1] + v)
        opt = _Options()
        L.pcv_default_options(ctypes.byref(opt))
        opt.device = self.device.index if self.device.index is not None else torch.cuda.current_device()
        opt.stream = _stream_ptr(stream).value
        opt.precision = FP64 if self.dtype == torch.float64 else FP32
        opt.use_graph = 1 if use_graph else 0
        b = ctypes.c_void_p()
        st = L.pcv_batch_create(ctypes.byref(b), ctypes.byref(opt))
        if st != 0:
            raise PcvError(st, "pcv_batch_create")
        self._b = b
        flat = torch.cat([t.contiguous().reshape(-1) for t in landmarks])
        na = (ctypes.c_int * self.W)(*self.n)
        nl = (ctypes.c_int * self.W)(*self.Ls)
        lm = (ctypes.c_double * self.W)(*[float(v) for v in lams])
        self._check(L.pcv_batch_load(b, self.W, na, nl, _ptr(flat), lm))
        del flat
        cp = cache_path.encode() if cache_path else None
        self._check(L.pcv_batch_plan(b, 1 if tune else 0, cp))
        self.sz = torch.empty(self.W, 2, dtype=torch.float64, device=self.device)
        self.ds = torch.empty(self.atom_off[-1], 3, dtype=self.dtype, device=self.device)
        self.dz = torch.empty(self.atom_off[-1], 3, dtype=self.dtype, device=self.device)

    def _check(self, status):
        if status != 0:
            raise PcvError(status, (self._L.pcv_batch_last_error(self._b) or b"").decode())

    @property
    def plan(self) -> str:
        return (self._L.pcv_batch_plan_string(self._b) or b"").decode()

    def eval(self, x_all, *, grad: bool = True):
        """``x_all``: CUDA tensor ``[sum n_w][3]``.  Returns (sz [W][2], ds, dz)."""
        if not (x_all.is_cuda and x_all.dtype == self.dtype and tuple(x_all.shape) == (self.atom_off[-1], 3)
                and x_all.is_contiguous()):
            raise ValueError("x_all must be a contiguous CUDA tensor [sum n_w][3] of the landmark dtype")
        self._check(self._L.pcv_batch_eval(self._b, _ptr(x_all), _ptr(self.sz),
                                           _ptr(self.ds) if grad else None, _ptr(self.dz) if grad else None))
        return self.sz, self.ds, self.dz

    def set_kernel_timing(self, enable: bool):
        """HIP-event timing of the landmark streaming launch (eager calls)."""
        self._check(self._L.pcv_batch_set_kernel_timing(self._b, int(bool(enable))))

    def kernel_timing(self):
        """(summed engine ms, launches) since timing was enabled."""
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        self._check(self._L.pcv_batch_get_kernel_timing(self._b, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "_b", None) is not None:
            self._L.pcv_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """MLP surrogate of (s, z) on one GPU (BF16 matrix-core kernels).

    ``ref``: host ``[n][3]`` reference the inputs are aligned to; ``hidden``:
    hidden width; ``max_batch``: largest batch of any call.  Parameters are
    one flat FP32 array (W_l [fan_in][fan_out] then b_l, l = 1..4) supplied by
    the caller (``set_params``).
    """

    def __init__(self, ref, *, hidden: int = 512, max_batch: int = 1024, w=None, use_graph: bool = False,
                 stream=None, device: int = 0):
        import numpy as np
        self._L = load_library()
        ref = np.ascontiguousarray(np.asarray(ref, dtype=np.float64))
        self.n = ref.shape[0]
        self.hidden = hidden
        self.max_batch = max_batch
        opt = _Options()
        self._L.pcv_default_options(ctypes.byref(opt))
        opt.device = device
        opt.precision = FP32
        opt.use_graph = 1 if use_graph else 0
        opt.stream = _stream_ptr(stream)
        warr, wptr = _as_host_f64(w, self.n, "w")
        self._keep = (ref, warr)
        h = ctypes.c_void_p()
        s = self._L.pcv_mlp_create(ctypes.byref(h), ctypes.byref(opt), self.n, hidden, max_batch,
                                   ref.ctypes.data_as(ctypes.c_void_p), wptr)
        if s != 0:
            raise PcvError(s, self._L.pcv_status_string(s).decode())
        self._h = h
        self.param_count = int(self._L.pcv_mlp_param_count(h))

    def _check(self, s):
        if s != 0:
            msg = self._L.pcv_mlp_last_error(self._h).decode()
            raise PcvError(s, f"{self._L.pcv_status_string(s).decode()}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.pcv_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if p.size != self.param_count:
            raise ValueError(f"expected {self.param_count} parameters")
        self._check(self._L.pcv_mlp_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size))

    def params(self):
        import numpy as np
        p = np.empty(self.param_count, dtype=np.float32)
        self._check(self._L.pcv_mlp_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size))
        return p

    def grads(self):
        import numpy as np
        p = np.empty(self.param_count, dtype=np.float32)
        self._check(self._L.pcv_mlp_get_grads(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size))
        return p

    def set_scaling(self, mean, sd):
        import numpy as np
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float64))
        d = np.ascontiguousarray(np.asarray(sd, dtype=np.float64))
        self._keep_scaling = (m, d)
        self._check(self._L.pcv_mlp_set_scaling(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                                d.ctypes.data_as(ctypes.c_void_p)))

    def align(self, x, *, bf16: bool = True, f32: bool = False):
        """Aligned inputs of structures ``x`` (CUDA float32 ``[B][n][3]``):
        BF16 bits as int16 ``[B][3n]`` and/or float32."""
        import torch
        x = x.contiguous()
        B = x.shape[0]
        ob = torch.empty(B, 3 * self.n, dtype=torch.int16, device=x.device) if bf16 else None
        of = torch.empty(B, 3 * self.n, dtype=torch.float32, device=x.device) if f32 else None
        self._check(self._L.pcv_mlp_align(self._h, _ptr(x), B, _ptr(ob), _ptr(of)))
        return ob, of

    def forward(self, inputs):
        import torch
        B = inputs.shape[0]
        y = torch.empty(B, 2, dtype=torch.float32, device=inputs.device)
        self._check(self._L.pcv_mlp_forward(self._h, _ptr(inputs.contiguous()), B, _ptr(y)))
        return y

    def train_step(self, inputs, targets, lr: float, loss=None):
        """One Adam step on BF16 inputs ``[B][3n]`` (int16 bits) and float32
        standardised targets ``[B][2]``; ``loss`` (float32 tensor [1]) receives
        the loss before the step."""
        self._check(self._L.pcv_mlp_train_step(self._h, _ptr(inputs), _ptr(targets), inputs.shape[0],
                                               ctypes.c_float(lr), _ptr(loss)))

    def eval(self, x, *, grad: bool = True, out=None):
        """(s, z) and gradients for raw structures ``x`` ``[B][n][3]`` (float32)."""
        import torch
        x = x.contiguous()
        B = x.shape[0]
        o = out or {}
        sz = o.get("sz") if o.get("sz") is not None else torch.empty(B, 2, dtype=torch.float64, device=x.device)
        ds = dz = None
        if grad:
            ds = o.get("ds_dx") if o.get("ds_dx") is not None else torch.empty_like(x)
            dz = o.get("dz_dx") if o.get("dz_dx") is not None else torch.empty_like(x)
        self._check(self._L.pcv_mlp_eval(self._h, _ptr(x), B, _ptr(sz), _ptr(ds), _ptr(dz)))
        return {"sz": sz, "ds_dx": ds, "dz_dx": dz}

    def step(self, exact: "PathCV", x, *, out=None):
        """One fallback step (drift test of the exact handle ``exact``)."""
        import torch
        o = out or {}
        sz = o.get("sz") if o.get("sz") is not None else torch.empty(2, dtype=torch.float64, device=x.device)
        ds = o.get("ds_dx") if o.get("ds_dx") is not None else torch.empty_like(x)
        dz = o.get("dz_dx") if o.get("dz_dx") is not None else torch.empty_like(x)
        used = o.get("used") if o.get("used") is not None else torch.empty(1, dtype=torch.int32, device=x.device)
        self._check(self._L.pcv_mlp_step(self._h, exact._h, _ptr(x), _ptr(sz), _ptr(ds), _ptr(dz), _ptr(used)))
        return {"sz": sz, "ds_dx": ds, "dz_dx": dz, "used": used}

    def save_state(self) -> bytes:
        """Training state (parameters, Adam moments and step, scaling, the
        fallback anchor) as bytes (``pcv_mlp_save_state``)."""
        n = ctypes.c_size_t(0)
        self._check(self._L.pcv_mlp_save_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._L.pcv_mlp_save_state(self._h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def load_state(self, blob: bytes):
        """Restore a state written by ``save_state`` (``pcv_mlp_load_state``)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(self._L.pcv_mlp_load_state(self._h, buf, len(blob)))

    def stats(self) -> dict:
        st = _MlpStats()
        self._check(self._L.pcv_mlp_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _MlpStats._fields_}

    def reset_stats(self):
        self._check(self._L.pcv_mlp_reset_stats(self._h))


class Bias:
    """Metadynamics bias of Eq. 1 on (s, z), kept on a device grid.

    ``s_range``, ``z_range``: (min, max); ``bins``: (ns, nz) nodes;
    ``height`` and ``sigma`` = (sigma_s, sigma_z) of every hill.
    """

    def __init__(self, s_range, z_range, bins, height: float, sigma, *, stream=None, device: int = 0):
        self._L = load_library()
        o = _BiasOptions()
        o.device = device
        o.stream = _stream_ptr(stream)
        o.s_min, o.s_max = float(s_range[0]), float(s_range[1])
        o.z_min, o.z_max = float(z_range[0]), float(z_range[1])
        o.ns, o.nz = int(bins[0]), int(bins[1])
        o.height = float(height)
        o.sigma_s, o.sigma_z = float(sigma[0]), float(sigma[1])
        self.shape = (o.ns, o.nz)
        h = ctypes.c_void_p()
        st = self._L.pcv_bias_create(ctypes.byref(h), ctypes.byref(o))
        if st != 0:
            raise PcvError(st, self._L.pcv_status_string(st).decode())
        self._h = h

    def _check(self, s):
        if s != 0:
            msg = self._L.pcv_bias_last_error(self._h).decode()
            raise PcvError(s, f"{self._L.pcv_status_string(s).decode()}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.pcv_bias_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def deposit(self, sz):
        """One hill at the CV values of the device tensor ``sz`` (float64 [2])."""
        self._check(self._L.pcv_bias_deposit(self._h, _ptr(sz)))

    def gradient(self, sz, ds_dx=None, dz_dx=None, *, out=None):
        """Bias (V, dV/ds, dV/dz) at ``sz`` and dV/dx (same dtype as ds_dx).
        Returns (grad or None, v [3] float64, in_range [1] int32), all device tensors."""
        import torch
        o = out or {}
        v = o.get("v") if o.get("v") is not None else torch.empty(3, dtype=torch.float64, device=sz.device)
        ok = o.get("in_range") if o.get("in_range") is not None else torch.empty(1, dtype=torch.int32,
                                                                                 device=sz.device)
        grad = None
        n, prec = 0, FP32
        if ds_dx is not None:
            if dz_dx is None or ds_dx.shape != dz_dx.shape or ds_dx.dtype != dz_dx.dtype:
                raise ValueError("ds_dx and dz_dx must match")
            n = ds_dx.shape[0]
            prec = FP64 if ds_dx.dtype == torch.float64 else FP32
            grad = o.get("grad") if o.get("grad") is not None else torch.empty_like(ds_dx)
        self._check(self._L.pcv_bias_gradient(self._h, _ptr(sz), n, prec, _ptr(ds_dx), _ptr(dz_dx), _ptr(grad),
                                              _ptr(v), _ptr(ok)))
        return grad, v, ok

    def hills(self) -> int:
        c = ctypes.c_longlong()
        self._check(self._L.pcv_bias_hills(self._h, ctypes.byref(c)))
        return c.value

    def grid(self):
        """Host copy [4][ns][nz]: V, dV/ds, dV/dz, d2V/dsdz at the nodes."""
        import numpy as np
        out = np.empty((4,) + self.shape, dtype=np.float64)
        self._check(self._L.pcv_bias_get_grid(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out


def stream_read(buf, wg_sums, grid: int, stream=None):
    """Read the CUDA tensor ``buf`` once with the engines' load path (the
    streaming-read ceiling, ``pcv_stream_read``); per-workgroup float sums go
    to ``wg_sums`` (float64 [grid])."""
    import torch
    if not (buf.is_cuda and buf.is_contiguous() and wg_sums.is_cuda and wg_sums.dtype == torch.float64
            and wg_sums.numel() >= grid):
        raise ValueError("buf: contiguous CUDA tensor; wg_sums: CUDA float64 tensor of at least grid entries")
    L = load_library()
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    s = L.pcv_stream_read(_ptr(buf), buf.numel() * buf.element_size(), _ptr(wg_sums), grid, st)
    if s != 0:
        raise PcvError(s, L.pcv_status_string(s).decode())
