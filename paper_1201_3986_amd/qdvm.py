"""Python binding of libqdvm (ctypes): argument marshalling only.

Every step of the collision operator runs in the HIP library; this module
checks tensor shapes, passes device pointers and the current HIP stream, and
maps status codes to exceptions.  PyTorch provides device memory and streams.
If the built library is missing, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libqdvm.so")

QDVM_OK, QDVM_EINVAL, QDVM_EUNSUPPORTED, QDVM_ENOMEM, QDVM_EDEVICE = 0, -1, -2, -3, -4
MODE_FULL, MODE_NEAR_EQUILIBRIUM = 0, 1
LINE_UNIFORM, LINE_DELTA = 0, 1
_LINE_WEIGHTS = {"uniform": LINE_UNIFORM, "delta": LINE_DELTA}
ABI_VERSION = 4
_MODES = {"full": MODE_FULL, "near_equilibrium": MODE_NEAR_EQUILIBRIUM}

_lock = threading.Lock()
_lib = None


class QdvmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("qdvm status %d: %s" % (status, message))
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("half_width", ctypes.c_double),
                ("ntilde", ctypes.c_int32), ("farey_order", ctypes.c_int32), ("num_dirs", ctypes.c_int32),
                ("dirs", ctypes.POINTER(ctypes.c_int32)), ("weights", ctypes.POINTER(ctypes.c_double)),
                ("mode", ctypes.c_int32), ("line_weight", ctypes.c_int32)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("radix", ctypes.c_int32), ("threads", ctypes.c_int32), ("split", ctypes.c_int32),
                ("grid_div", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("ntilde", ctypes.c_int32),
                ("num_dirs", ctypes.c_int32), ("num_jobs", ctypes.c_int32), ("h", ctypes.c_double),
                ("mode", ctypes.c_int32), ("line_weight", ctypes.c_int32)]


def load():
    """Load libqdvm.so from the package's build folder (raises if absent)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError("libqdvm.so is not built (%s); run python -m paper_1201_3986_amd.build" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i32p, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), \
            ctypes.POINTER(ctypes.c_double)
        sigs = {
            "qdvm_plan": [ctypes.POINTER(Desc), ctypes.POINTER(vp)],
            "qdvm_plan_destroy": [vp],
            "qdvm_plan_info": [vp, ctypes.POINTER(PlanInfo)],
            "qdvm_plan_dirs": [vp, i32p, dp, i32p],
            "qdvm_describe": [ctypes.POINTER(Desc), i32p, i32p, dp, i32p, i32],
            "qdvm_eval": [vp, i32, vp, vp, vp, ctypes.c_float, vp],
            "qdvm_vjp": [vp, i32, vp, vp, vp, vp, vp, vp],
            "qdvm_eval_noalloc": [vp, i32, vp, vp, vp, ctypes.c_float, vp],
            "qdvm_eval_bilinear": [vp, i32, vp, vp, vp, vp, ctypes.c_float, vp],
            "qdvm_transform_stage": [i32, i32, i32, i32, i32, vp, vp, vp],
            "qdvm_eval_pseudo_spectral": [vp, i32, vp, vp, vp],
            "qdvm_set_variant": [vp, i32, i32],
            "qdvm_get_variant": [vp, i32, i32p],
            "qdvm_autotune": [vp, i32, vp],
            "qdvm_set_config": [vp, i32, ctypes.POINTER(LaunchConfig)],
            "qdvm_get_config": [vp, i32, ctypes.POINTER(LaunchConfig)],
            "qdvm_batch_plan": [i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(vp)],
            "qdvm_batch_destroy": [vp],
            "qdvm_batch_info": [vp, i32p, i32p, dp],
            "qdvm_batch_eval": [vp, vp, vp, ctypes.c_float, vp],
            "qdvm_eval_batched": [i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64), vp, vp, ctypes.c_float, vp],
            "qdvm_step_graph_create": [vp, vp, ctypes.c_float, vp, ctypes.POINTER(vp)],
            "qdvm_step_graph_create_scheme": [vp, vp, ctypes.c_float, i32, vp, ctypes.POINTER(vp)],
            "qdvm_step_graph_launch": [vp, vp],
            "qdvm_step_graph_destroy": [vp],
            "qdvm_adaptive_plan": [i32, ctypes.POINTER(ctypes.c_int64), i32, ctypes.POINTER(vp),
                                   ctypes.POINTER(ctypes.c_float), ctypes.POINTER(vp)],
            "qdvm_adaptive_eval": [vp, vp, vp, ctypes.c_float, vp, vp, vp],
            "qdvm_adaptive_destroy": [vp],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.qdvm_status_string.argtypes = [ctypes.c_int]
        lib.qdvm_status_string.restype = ctypes.c_char_p
        lib.qdvm_last_error.restype = ctypes.c_char_p
        lib.qdvm_abi_version.restype = ctypes.c_int32
        lib.qdvm_noalloc_scratch_bytes.restype = ctypes.c_size_t
        if lib.qdvm_abi_version() != ABI_VERSION:
            raise ImportError("libqdvm.so has ABI %d, the binding expects %d; rebuild it"
                              % (lib.qdvm_abi_version(), ABI_VERSION))
        _lib = lib
        return lib


def _check(status: int):
    if status != QDVM_OK:
        lib = load()
        raise QdvmError(status, lib.qdvm_last_error().decode() or lib.qdvm_status_string(status).decode())


def _mode(mode):
    if isinstance(mode, str):
        if mode not in _MODES:
            raise ValueError("mode must be one of %s" % sorted(_MODES))
        return _MODES[mode]
    return int(mode)


def _line_weight(lw):
    if isinstance(lw, str):
        if lw not in _LINE_WEIGHTS:
            raise ValueError("line_weight must be one of %s" % sorted(_LINE_WEIGHTS))
        return _LINE_WEIGHTS[lw]
    return int(lw)


def _desc(dim, n, half_width, ntilde, farey_order, num_dirs, dirs, weights, mode=MODE_FULL, line_weight=LINE_UNIFORM):
    keep = []
    d = Desc(dim, n, float(half_width), ntilde, farey_order, num_dirs, None, None, _mode(mode),
             _line_weight(line_weight))
    if dirs is not None:
        a = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1, dim))
        keep.append(a)
        d.dirs = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.num_dirs = a.shape[0]
    if weights is not None:
        wv = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        keep.append(wv)
        d.weights = wv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d, keep


def describe(dim, n, half_width=8.0, ntilde=0, farey_order=0, num_dirs=0, dirs=None, weights=None,
             line_weight=LINE_UNIFORM):
    """Host-only: (dirs, weights, line lengths) a descriptor selects."""
    lib = load()
    d, keep = _desc(dim, n, half_width, ntilde, farey_order, num_dirs, dirs, weights, line_weight=line_weight)
    P = ctypes.c_int32(0)
    _check(lib.qdvm_describe(ctypes.byref(d), ctypes.byref(P), None, None, None, 0))
    dirs_out = np.zeros((P.value, dim), dtype=np.int32)
    w_out = np.zeros(P.value, dtype=np.float64)
    m_out = np.zeros(P.value, dtype=np.int32)
    _check(lib.qdvm_describe(ctypes.byref(d), ctypes.byref(P),
                             dirs_out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             w_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             m_out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), P.value))
    return dirs_out, w_out, m_out


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Plan:
    """An immutable plan (directions, weights, multiplier tables) on the current device."""

    def __init__(self, dim, n, half_width=8.0, ntilde=0, farey_order=0, num_dirs=0, dirs=None, weights=None,
                 mode=MODE_FULL, line_weight=LINE_UNIFORM):
        """mode: "full" (Q(f, f)) or "near_equilibrium" (Q(f, f) - Q(M, M) with M
        the cell's Maxwellian, evaluated as Q(g, f) + Q(M, g), g = f - M).
        line_weight: "uniform" (a(m e_p) = w_p, the paper's lattice weights) or
        "delta" (a(m e_p) = w_p / |m|, the quadrature of delta(x . y))."""
        lib = load()
        d, keep = _desc(dim, n, half_width, ntilde, farey_order, num_dirs, dirs, weights, mode, line_weight)
        h = ctypes.c_void_p()
        _check(lib.qdvm_plan(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        # what the caller asked for (explicit lists or the defaults the library fills in)
        self.request = dict(half_width=float(half_width), ntilde=int(ntilde), farey_order=int(farey_order),
                            num_dirs=int(num_dirs), explicit_dirs=dirs is not None,
                            explicit_weights=weights is not None)
        self.line_weight = _line_weight(line_weight)
        info = PlanInfo()
        _check(lib.qdvm_plan_info(h, ctypes.byref(info)))
        self.dim, self.n, self.ntilde = info.dim, info.n, info.ntilde
        self.num_dirs, self.num_jobs, self.h = info.num_dirs, info.num_jobs, info.h
        self.mode = info.mode
        self.npts = self.n ** self.dim
        self.dirs = np.zeros((self.num_dirs, dim), dtype=np.int32)
        self.weights = np.zeros(self.num_dirs, dtype=np.float64)
        self.line_len = np.zeros(self.num_dirs, dtype=np.int32)
        _check(lib.qdvm_plan_dirs(h, self.dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  self.weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  self.line_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().qdvm_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _cells(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
            raise TypeError("%s must be a float32 CUDA tensor" % name)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if t.numel() % self.npts:
            raise ValueError("%s has %d elements, not a multiple of n^d = %d" % (name, t.numel(), self.npts))
        return t.numel() // self.npts

    def _weights(self, w):
        import torch
        if w is None:
            return None
        if not w.is_cuda or w.dtype != torch.float32 or w.numel() != self.num_dirs or not w.is_contiguous():
            raise ValueError("w must be a contiguous float32 CUDA tensor of %d weights" % self.num_dirs)
        return w

    def eval(self, f, out=None, w=None, dt=0.0, stream=None):
        """Q(f, f) (dt == 0) or f + dt Q(f, f) for every cell of f; out may be f."""
        import torch
        batch = self._cells(f, "f")
        if out is None:
            out = torch.empty_like(f)
        elif self._cells(out, "out") != batch:
            raise ValueError("out and f differ in size")
        w = self._weights(w)
        _check(load().qdvm_eval(self._h, batch, _ptr(f), _ptr(out), _ptr(w), float(dt), _stream_ptr(stream)))
        return out

    def eval_bilinear(self, g, f, out=None, w=None, dt=0.0, stream=None):
        """Q(g, f) (dt == 0) or g + dt Q(g, f) for every cell; out may be g or f."""
        import torch
        batch = self._cells(g, "g")
        if self._cells(f, "f") != batch:
            raise ValueError("g and f differ in size")
        if out is None:
            out = torch.empty_like(g)
        elif self._cells(out, "out") != batch:
            raise ValueError("out and g differ in size")
        w = self._weights(w)
        _check(load().qdvm_eval_bilinear(self._h, batch, _ptr(g), _ptr(f), _ptr(out), _ptr(w), float(dt),
                                         _stream_ptr(stream)))
        return out

    def eval_pseudo_spectral(self, f, out=None, stream=None):
        """Q(f, f) by the O(n^2d) pseudo-spectral form in FP64 (2D n <= 32, 3D n = 8)."""
        import torch
        batch = self._cells(f, "f")
        if out is None:
            out = torch.empty_like(f)
        elif self._cells(out, "out") != batch:
            raise ValueError("out and f differ in size")
        _check(load().qdvm_eval_pseudo_spectral(self._h, batch, _ptr(f), _ptr(out), _stream_ptr(stream)))
        return out

    def eval_noalloc(self, f, out, w=None, dt=0.0, stream=None):
        """As eval, through qdvm_eval_noalloc: the launch's scratch is the
        library's static device array (nothing is allocated); out is required."""
        batch = self._cells(f, "f")
        if self._cells(out, "out") != batch:
            raise ValueError("out and f differ in size")
        w = self._weights(w)
        _check(load().qdvm_eval_noalloc(self._h, batch, _ptr(f), _ptr(out), _ptr(w), float(dt),
                                        _stream_ptr(stream)))
        return out

    def vjp(self, f, cot, w=None, want_grad_w=True, stream=None):
        """(grad_f, grad_w) of <cot, Q(f; w)>, grad_w summed over the cells."""
        import torch
        batch = self._cells(f, "f")
        if self._cells(cot, "cot") != batch:
            raise ValueError("cot and f differ in size")
        w = self._weights(w)
        gf = torch.empty_like(f)
        gw = torch.empty(self.num_dirs, dtype=torch.float32, device=f.device) if want_grad_w else None
        _check(load().qdvm_vjp(self._h, batch, _ptr(f), _ptr(cot), _ptr(w), _ptr(gf), _ptr(gw),
                               _stream_ptr(stream)))
        return gf, gw

    def set_variant(self, op: int, variant: int):
        _check(load().qdvm_set_variant(self._h, op, variant))

    def get_variant(self, op: int) -> int:
        v = ctypes.c_int32(0)
        _check(load().qdvm_get_variant(self._h, op, ctypes.byref(v)))
        return v.value

    def autotune(self, batch: int, stream=None):
        """Time the launch shapes of evaluation and adjoint on `batch` cells and
        keep the fastest (cached in the file $QDVM_TUNE_CACHE names, if set)."""
        _check(load().qdvm_autotune(self._h, batch, _stream_ptr(stream)))

    def set_config(self, op: int, radix=-1, threads=0, split=0, grid_div=1):
        """Launch shape of op 0 (evaluation) or 1 (adjoint); no arguments: defaults."""
        c = LaunchConfig(radix, threads, split, grid_div)
        _check(load().qdvm_set_config(self._h, op, ctypes.byref(c)))

    def get_config(self, op: int) -> dict:
        c = LaunchConfig()
        _check(load().qdvm_get_config(self._h, op, ctypes.byref(c)))
        return dict(radix=c.radix, threads=c.threads, split=c.split, grid_div=c.grid_div)


def _plan_array(plans):
    arr = (ctypes.c_void_p * len(plans))()
    for i, p in enumerate(plans):
        arr[i] = p.handle.value
    return arr


class BatchPlan:
    """Heterogeneous batch: cell i uses plans[i] and lives at f[offsets[i] : offsets[i] + n_i^d]."""

    def __init__(self, plans, offsets):
        lib = load()
        self._plans = list(plans)            # plans must outlive the batch
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if len(self._plans) != len(self.offsets):
            raise ValueError("plans and offsets differ in length")
        self.extent = int(max((o + p.npts for p, o in zip(self._plans, self.offsets)), default=0))
        h = ctypes.c_void_p()
        _check(lib.qdvm_batch_plan(len(self._plans), _plan_array(self._plans),
                                   self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(h)))
        self._h = h
        la, it, fl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib.qdvm_batch_info(h, ctypes.byref(la), ctypes.byref(it), ctypes.byref(fl)))
        self.launches, self.items, self.flops = la.value, it.value, fl.value

    @property
    def handle(self):
        return self._h

    def _check_buf(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError("%s must be a contiguous float32 CUDA tensor" % name)
        if t.numel() < self.extent:
            raise ValueError("%s has %d elements, the batch addresses %d" % (name, t.numel(), self.extent))

    def eval(self, f, out=None, dt=0.0, stream=None):
        import torch
        self._check_buf(f, "f")
        if out is None:
            out = torch.empty_like(f)
        self._check_buf(out, "out")
        _check(load().qdvm_batch_eval(self._h, _ptr(f), _ptr(out), float(dt), _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().qdvm_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AdaptivePlan(BatchPlan):
    """Cells of one grid size, each evaluated with the plan of its level:
    level l when the cell's distance from its Maxwellian, sum|f - M| / sum|f|,
    exceeds l of the increasing `thresholds` (len(level_plans) - 1 values).
    The levels are chosen on the device at every evaluation."""

    def __init__(self, level_plans, offsets, thresholds):
        lib = load()
        self._plans = list(level_plans)      # plans must outlive the batch
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float32))
        if len(thr) != max(len(self._plans) - 1, 0):
            raise ValueError("need len(level_plans) - 1 thresholds")
        self.thresholds = thr
        npts = self._plans[0].npts if self._plans else 0
        self.npts = npts
        self.extent = int(self.offsets.max() + npts) if len(self.offsets) else 0
        h = ctypes.c_void_p()
        _check(lib.qdvm_adaptive_plan(len(self.offsets), self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      len(self._plans), _plan_array(self._plans),
                                      thr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h)))
        self._h = h

    def eval(self, f, out=None, dt=0.0, levels=False, stream=None):
        """Q per cell (or f + dt Q); with levels=True also returns each cell's
        level (int32) and distance from equilibrium (float32) as CUDA tensors."""
        import torch
        self._check_buf(f, "f")
        if out is None:
            out = torch.empty_like(f)
        self._check_buf(out, "out")
        lv = dist = None
        if levels:
            lv = torch.empty(len(self.offsets), dtype=torch.int32, device=f.device)
            dist = torch.empty(len(self.offsets), dtype=torch.float32, device=f.device)
        _check(load().qdvm_adaptive_eval(self._h, _ptr(f), _ptr(out), float(dt),
                                         _ptr(lv) if levels else None, _ptr(dist) if levels else None,
                                         _stream_ptr(stream)))
        return (out, lv, dist) if levels else out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().qdvm_adaptive_destroy(self._h))
            self._h = ctypes.c_void_p()


STEP_EULER, STEP_RK2 = 0, 1
_SCHEMES = {"euler": STEP_EULER, "rk2": STEP_RK2}


class StepGraph:
    """In-place time step of a batch, captured once into a HIP graph:
    scheme "euler" (f <- f + dt Q(f)) or "rk2" (the two-stage TVD Runge-Kutta
    step f1 = f + dt Q(f), f <- (f + f1 + dt Q(f1)) / 2)."""

    def __init__(self, batch: BatchPlan, f, dt, capture_stream, scheme="euler"):
        batch._check_buf(f, "f")
        if isinstance(scheme, str):
            if scheme not in _SCHEMES:
                raise ValueError("scheme must be one of %s" % sorted(_SCHEMES))
            scheme = _SCHEMES[scheme]
        self._batch, self._f = batch, f
        h = ctypes.c_void_p()
        _check(load().qdvm_step_graph_create_scheme(batch.handle, _ptr(f), float(dt), int(scheme),
                                                    ctypes.c_void_p(capture_stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(load().qdvm_step_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().qdvm_step_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_batched(plans, offsets, f, out, dt=0.0, stream=None):
    """One-shot heterogeneous evaluation (synchronises the stream)."""
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    _check(load().qdvm_eval_batched(len(plans), _plan_array(plans),
                                    offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    _ptr(f), _ptr(out), float(dt), _stream_ptr(stream)))
    return out


def transform_stage(f, method=0, reps=0, stream=None):
    """Forward 2D transform of n = 16 cells (f: float32 CUDA, batch * 256) as
    complex spectra out[cell][K1][K0] (complex64 CUDA tensor); method 0 the
    register FFT, 1 the matrix-core DFT; reps inverse-forward round trips in
    registers before the spectrum is written."""
    import torch
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32 or not f.is_contiguous():
        raise TypeError("f must be a contiguous float32 CUDA tensor")
    if f.numel() % 256:
        raise ValueError("f is not a whole number of 16 x 16 cells")
    batch = f.numel() // 256
    out = torch.empty(batch, 16, 16, dtype=torch.complex64, device=f.device)
    _check(load().qdvm_transform_stage(int(method), 2, 16, batch, int(reps), _ptr(f), _ptr(out),
                                       _stream_ptr(stream)))
    return out


def _make_function():
    import torch

    class QdvmFunction(torch.autograd.Function):
        """Q(f; w) with the hand-written adjoint as backward.

        forward(f, w, plan): f float32 CUDA (batch * n^d), w float32 CUDA (P) or None.
        """

        @staticmethod
        def forward(ctx, f, w, plan):
            ctx.plan = plan
            f = f.contiguous()
            w = w.contiguous() if w is not None else None
            ctx.save_for_backward(f, w if w is not None else torch.empty(0, device=f.device))
            ctx.has_w = w is not None
            return plan.eval(f, w=w)

        @staticmethod
        def backward(ctx, grad_out):
            f, w = ctx.saved_tensors
            w = w if ctx.has_w else None
            need_w = ctx.needs_input_grad[1]
            gf, gw = ctx.plan.vjp(f, grad_out.contiguous(), w=w, want_grad_w=need_w)
            return gf, (gw if need_w else None), None

    return QdvmFunction


_fn = None


def collide(f, plan: Plan, w=None):
    """Differentiable Q(f; w) through QdvmFunction."""
    global _fn
    if _fn is None:
        _fn = _make_function()
    return _fn.apply(f, w, plan)
