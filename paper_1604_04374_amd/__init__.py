"""Convolution-product expansions on MI355X: Python binding of ``libpc.so``.

The expansion of order ``m`` (eq. 1.4)

    H_m u = sum_k h_k * (w_k . u),      H_m^* v = sum_k w_k . (h~_k * v)

is evaluated by the HIP library behind the C ABI of ``include/pc.h``.  This
module only marshals arguments: host arrays (windows, impulse responses) are
passed as pointers at plan creation; signals are torch CUDA tensors whose
device pointers and the current HIP stream are handed to the library.  Every
step of the computation runs in the library's kernels; there is no other
implementation, and a missing library is an error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple, Union

import numpy as np

__all__ = ["Plan", "Batch", "PCError", "KernelStat", "TuneEntry", "TUNE_KNOBS", "load_tuning", "tune_set",
           "tune_key", "tune_batch_key", "tuning_table_path", "PC_PLAN_GRADIENTS", "PC_PLAN_PRODUCT_CONVOLUTION",
           "PC_PLAN_FULL_GRID", "PC_BATCH_NO_GRAPH", "PC_BATCH_PERSISTENT", "load_library", "LIB_PATH", "EXPORTS", "PlanDesc", "PlanInfo",
           "PC_W_DENSE", "PC_W_SEPARABLE", "construct_project", "construct_interpolate", "wavelet_transform"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpc.so")

PC_W_DENSE = 0
PC_W_SEPARABLE = 1

STATUS_NAMES = {
    0: "PC_SUCCESS",
    1: "PC_ERROR_INVALID_VALUE",
    2: "PC_ERROR_UNSUPPORTED",
    3: "PC_ERROR_OUT_OF_MEMORY",
    4: "PC_ERROR_HIP",
    5: "PC_ERROR_INVALID_PLAN",
}

# Every symbol include/pc.h declares.
EXPORTS = ("pc_plan_create", "pc_apply", "pc_apply_adjoint", "pc_destroy", "pc_plan_query",
           "pc_plan_set_spectra", "pc_plan_get_spectra", "pc_grad_spectra",
           "pc_plan_set_tracing", "pc_plan_trace_stats", "pc_plan_trace_reset",
           "pc_plan_set_responses", "pc_construct_project", "pc_construct_interpolate",
           "pc_wavelet_transform", "pc_wavelet_transform_noalloc", "pc_plan_create_meyer",
           "pc_batch_create", "pc_batch_apply", "pc_batch_apply_adjoint", "pc_batch_destroy",
           "pc_plan_sections", "pc_apply_save", "pc_backward", "pc_plan_set_budget",
           "pc_tune_set", "pc_tune_key", "pc_tune_batch_key",
           "pc_status_string", "pc_last_error")

PC_BATCH_NO_GRAPH = 1
PC_BATCH_PERSISTENT = 2

PC_PLAN_GRADIENTS = 1
PC_PLAN_PRODUCT_CONVOLUTION = 2
PC_PLAN_FULL_GRID = 4


class PlanDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("m", ctypes.c_int32), ("n0", ctypes.c_int64),
                ("n1", ctypes.c_int64), ("batch", ctypes.c_int64), ("w_format", ctypes.c_int32),
                ("m_rows", ctypes.c_int32), ("m_cols", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("fft_inner", ctypes.c_int32), ("fft_outer", ctypes.c_int32),
                ("n_items", ctypes.c_int32), ("spectra_bytes", ctypes.c_int64),
                ("window_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("keep_bytes", ctypes.c_int64), ("spectra_count", ctypes.c_int64)]


class SectionInfo(ctypes.Structure):
    _fields_ = [("term", ctypes.c_int32), ("m1", ctypes.c_int32), ("m2", ctypes.c_int32),
                ("win_o1", ctypes.c_int32), ("win_p1", ctypes.c_int32), ("win_o2", ctypes.c_int32),
                ("win_p2", ctypes.c_int32), ("lag_o1", ctypes.c_int32), ("lag_q1", ctypes.c_int32),
                ("lag_o2", ctypes.c_int32), ("lag_q2", ctypes.c_int32), ("spec_offset", ctypes.c_int64)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("key", ctypes.c_uint64), ("knob", ctypes.c_int32), ("length", ctypes.c_int32),
                ("value", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# knob names of the tuning table (include/pc.h PC_TUNE_*)
TUNE_KNOBS = {"cols_fwd_late": 1, "cols_adj_prefetch": 2, "rows_inv_pipe": 3, "rows_fwd_small": 4,
              "rows_inv_small": 5, "col_groups": 6, "fourstep_l": 7, "batch_persistent": 8, "sec_streams": 9,
              "keep": 10}
TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


class KernelStat(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


class PCError(RuntimeError):
    """A library call returned a status other than PC_SUCCESS."""

    def __init__(self, status: int, call: str, detail: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{call}: {self.name}: {detail}")


_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libpc.so`` (once) and declare its signatures."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_1604_04374_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.pc_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc), vp, vp, vp]
    lib.pc_plan_create.restype = ctypes.c_int
    for name in ("pc_apply", "pc_apply_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, i64, vp]
        f.restype = ctypes.c_int
    lib.pc_destroy.argtypes = [vp]
    lib.pc_destroy.restype = ctypes.c_int
    lib.pc_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.pc_plan_query.restype = ctypes.c_int
    lib.pc_plan_set_spectra.argtypes = [vp, vp, vp]
    lib.pc_plan_set_spectra.restype = ctypes.c_int
    lib.pc_plan_get_spectra.argtypes = [vp, vp, vp]
    lib.pc_plan_get_spectra.restype = ctypes.c_int
    lib.pc_grad_spectra.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.pc_grad_spectra.restype = ctypes.c_int
    lib.pc_plan_set_tracing.argtypes = [vp, ctypes.c_int32]
    lib.pc_plan_set_tracing.restype = ctypes.c_int
    lib.pc_plan_trace_stats.argtypes = [vp, ctypes.POINTER(KernelStat), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.pc_plan_trace_stats.restype = ctypes.c_int
    lib.pc_plan_trace_reset.argtypes = [vp]
    lib.pc_plan_trace_reset.restype = ctypes.c_int
    lib.pc_plan_sections.argtypes = [vp, ctypes.POINTER(SectionInfo), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.pc_plan_sections.restype = ctypes.c_int
    lib.pc_apply_save.argtypes = [vp, vp, vp, i64, vp]
    lib.pc_apply_save.restype = ctypes.c_int
    lib.pc_backward.argtypes = [vp, vp, vp, vp, vp, i64, ctypes.c_int32, vp]
    lib.pc_backward.restype = ctypes.c_int
    lib.pc_plan_set_budget.argtypes = [vp, i64]
    lib.pc_plan_set_budget.restype = ctypes.c_int
    lib.pc_tune_set.argtypes = [ctypes.POINTER(TuneEntry), ctypes.c_int32]
    lib.pc_tune_set.restype = ctypes.c_int
    lib.pc_tune_key.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_uint64)]
    lib.pc_tune_key.restype = ctypes.c_int
    lib.pc_tune_batch_key.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]
    lib.pc_tune_batch_key.restype = ctypes.c_int
    lib.pc_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp), ctypes.c_uint32, vp]
    lib.pc_batch_create.restype = ctypes.c_int
    for name in ("pc_batch_apply", "pc_batch_apply_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        f.restype = ctypes.c_int
    lib.pc_batch_destroy.argtypes = [vp]
    lib.pc_batch_destroy.restype = ctypes.c_int
    lib.pc_plan_set_responses.argtypes = [vp, vp, vp]
    lib.pc_plan_set_responses.restype = ctypes.c_int
    lib.pc_construct_project.argtypes = [i64, ctypes.c_int32, i64, vp, vp, vp, vp, vp]
    lib.pc_construct_project.restype = ctypes.c_int
    lib.pc_construct_interpolate.argtypes = [i64, ctypes.c_int32, i64, vp, vp, vp, vp, vp, vp]
    lib.pc_construct_interpolate.restype = ctypes.c_int
    lib.pc_wavelet_transform.argtypes = [ctypes.c_int32, i64, ctypes.c_int32, ctypes.c_int32, vp, i64, i64, i64,
                                         vp, vp, vp]
    lib.pc_wavelet_transform.restype = ctypes.c_int
    lib.pc_wavelet_transform_noalloc.argtypes = [ctypes.c_int32, i64, ctypes.c_int32, ctypes.c_int32, vp, i64, i64, i64,
                                         vp, vp, vp]
    lib.pc_wavelet_transform_noalloc.restype = ctypes.c_int
    lib.pc_plan_create_meyer.argtypes = [ctypes.POINTER(vp), i64, ctypes.c_int32, ctypes.c_int32, vp, i64, vp, vp,
                                         vp, i64, ctypes.c_uint32, vp]
    lib.pc_plan_create_meyer.restype = ctypes.c_int
    lib.pc_status_string.argtypes = [ctypes.c_int]
    lib.pc_status_string.restype = ctypes.c_char_p
    lib.pc_last_error.argtypes = []
    lib.pc_last_error.restype = ctypes.c_char_p
    if path == LIB_PATH:
        _lib = lib
        _load_default_tuning(lib)
    return lib


def _device_arch() -> Optional[str]:
    """gfx name of device 0, or None without a GPU (no device call is made
    when torch sees none)."""
    try:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return None


def tuning_table_path(arch: str) -> str:
    return os.path.join(TUNING_DIR, f"{arch}.json")


def _load_default_tuning(lib):
    arch = _device_arch()
    if arch is None:
        return
    path = tuning_table_path(arch)
    if os.path.exists(path):
        load_tuning(path, lib)


def load_tuning(path: str, lib=None) -> int:
    """Load a tuning table written by the tuner (JSON) into the library;
    returns the number of entries.  Plans and batches created afterwards use
    it."""
    import json
    with open(path) as fh:
        table = json.load(fh)
    entries = [(int(e["key"], 16), TUNE_KNOBS[e["knob"]], int(e["length"]), int(e["value"]))
               for e in table.get("entries", [])]
    tune_set(entries, lib)
    return len(entries)


def tune_set(entries, lib=None):
    """Replace the library's tuning table by (key, knob, length, value)
    tuples (knob: a PC_TUNE_* number); an empty list clears it."""
    lib = lib or load_library()
    n = len(entries)
    arr = (TuneEntry * max(n, 1))(*[TuneEntry(k, kn, ln, v, 0) for k, kn, ln, v in entries])
    _check(lib, lib.pc_tune_set(arr, n), "pc_tune_set")


def tune_key(desc) -> int:
    """Workload key of a plan description (PlanDesc)."""
    lib = load_library()
    k = ctypes.c_uint64()
    _check(lib, lib.pc_tune_key(ctypes.byref(desc), ctypes.byref(k)), "pc_tune_key")
    return k.value


def tune_batch_key(plans) -> int:
    """Workload key of a batch of plans."""
    lib = load_library()
    n = len(plans)
    hp = (ctypes.c_void_p * n)(*[p._handle.value for p in plans])
    k = ctypes.c_uint64()
    _check(lib, lib.pc_tune_batch_key(n, hp, ctypes.byref(k)), "pc_tune_batch_key")
    return k.value


def _check(lib, status: int, call: str):
    if status != 0:
        raise PCError(status, call, lib.pc_last_error().decode(errors="replace"))


def _stream_ptr(stream, device=None) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


class Plan:
    """The operator ``H_m`` of eq. 1.4 resident on the current device, or
    with ``product_convolution=True`` the product-convolution operator
    ``G_m u = sum_k w_k . (h_k * u)`` of eq. 1.3.

    Parameters
    ----------
    windows : array ``m x N`` / ``m x N1 x N2`` (dense), or a pair
        ``(a, b)`` of row-axis factors ``a`` (``m1 x N1``) and column-axis
        factors ``b`` (``m2 x N2``) for the separable grid
        ``w_{k1*m2+k2} = a_k1 (x) b_k2``.
    h : array ``m x N`` / ``m x N1 x N2``, impulse responses in lag layout.
    batch : largest number of signals per call.
    gradients : allocate the workspace of :meth:`grad_spectra` and
        :meth:`backward` (and keep windowed spectra within the budget).
    product_convolution : build ``G_m`` (eq. 1.3) instead of ``H_m``.
    full_grid : 2D: never evaluate section by section (sectioned plans,
        ``info()["path"] == 3``, take their sections' spectra as parameters;
        see :meth:`sections`).
    """

    def __init__(self, windows: Union[np.ndarray, Tuple[np.ndarray, np.ndarray]], h: np.ndarray,
                 batch: int = 1, stream=None, gradients: bool = False, product_convolution: bool = False,
                 full_grid: bool = False):
        self._lib = load_library()
        self._handle = ctypes.c_void_p()
        h = _f32(h)
        d = PlanDesc()
        d.m = h.shape[0]
        d.batch = int(batch)
        d.flags = ((PC_PLAN_GRADIENTS if gradients else 0) | (PC_PLAN_PRODUCT_CONVOLUTION if product_convolution else 0)
                   | (PC_PLAN_FULL_GRID if full_grid else 0))
        self.product_convolution = bool(product_convolution)
        if isinstance(windows, (tuple, list)):
            a, b = _f32(windows[0]), _f32(windows[1])
            d.w_format = PC_W_SEPARABLE
            d.m_rows, d.m_cols = a.shape[0], b.shape[0]
            wbuf = np.ascontiguousarray(np.concatenate([a.ravel(), b.ravel()]))
        else:
            wbuf = _f32(windows)
            d.w_format = PC_W_DENSE
            d.m_rows = d.m_cols = 0
        if h.ndim == 2:
            d.ndim, d.n0, d.n1 = 1, h.shape[1], 1
            self.shape = (int(h.shape[1]),)
        elif h.ndim == 3:
            d.ndim, d.n0, d.n1 = 2, h.shape[1], h.shape[2]
            self.shape = (int(h.shape[1]), int(h.shape[2]))
        else:
            raise ValueError("h must be m x N or m x N1 x N2")
        self.m = int(d.m)
        self.batch = int(batch)
        self.desc = d
        self._wbuf, self._hbuf = wbuf, h  # keep alive for the call
        s = _stream_ptr(stream)
        st = self._lib.pc_plan_create(ctypes.byref(self._handle), ctypes.byref(d),
                                      wbuf.ctypes.data_as(ctypes.c_void_p),
                                      h.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(s))
        _check(self._lib, st, "pc_plan_create")
        del self._wbuf, self._hbuf

    # ------------------------------------------------------------------
    def _prep(self, x, out):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32):
            raise TypeError("signals must be float32 CUDA tensors")
        x = x.contiguous()
        single = tuple(x.shape) == self.shape
        batch = 1 if single else int(x.shape[0])
        if not single and tuple(x.shape[1:]) != self.shape:
            raise ValueError(f"expected shape {self.shape} or (B, *{self.shape}), got {tuple(x.shape)}")
        if out is None:
            out = torch.empty_like(x)
        elif not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.shape == x.shape):
            raise ValueError("out must be a contiguous float32 CUDA tensor shaped like the input")
        return x, out, batch

    def apply(self, u, out=None, stream=None):
        """``y = H_m u`` (enqueued on ``stream``, default the current stream)."""
        u, out, batch = self._prep(u, out)
        st = self._lib.pc_apply(self._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                batch, ctypes.c_void_p(_stream_ptr(stream, u.device)))
        _check(self._lib, st, "pc_apply")
        return out

    def apply_save(self, u, out=None, stream=None):
        """:meth:`apply` that leaves in the plan what :meth:`backward` needs
        (pc_apply_save)."""
        u, out, batch = self._prep(u, out)
        st = self._lib.pc_apply_save(self._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     batch, ctypes.c_void_p(_stream_ptr(stream, u.device)))
        _check(self._lib, st, "pc_apply_save")
        return out

    def backward(self, u, gy, want_u=True, want_spectra=True, use_saved=False, stream=None):
        """(dL/du, dL/dspec) for y = H_m u and gy = dL/dy (pc_backward); either
        may be skipped (None).  ``use_saved``: u is unchanged since the last
        :meth:`apply` / :meth:`apply_save` on this plan."""
        import torch
        u, _, batch = self._prep(u, None)
        gy = gy.contiguous()
        if gy.shape != u.shape or gy.dtype != torch.float32 or not gy.is_cuda:
            raise ValueError("gy must be a float32 CUDA tensor shaped like u")
        gu = torch.empty_like(u) if want_u else None
        gs = torch.empty(self.spectra_shape, dtype=torch.complex64, device=u.device) if want_spectra else None
        st = self._lib.pc_backward(self._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                   ctypes.c_void_p(gu.data_ptr() if gu is not None else None),
                                   ctypes.c_void_p(gs.data_ptr() if gs is not None else None), batch,
                                   1 if use_saved else 0, ctypes.c_void_p(_stream_ptr(stream, u.device)))
        _check(self._lib, st, "pc_backward")
        return gu, gs

    def set_budget(self, nbytes: int):
        """Device bytes the plan may hold to keep the windowed spectra for
        :meth:`backward` (pc_plan_set_budget)."""
        _check(self._lib, self._lib.pc_plan_set_budget(self._handle, int(nbytes)), "pc_plan_set_budget")

    def sections(self) -> list:
        """The sections of a sectioned plan (pc_plan_sections), as dicts."""
        n = ctypes.c_int32()
        _check(self._lib, self._lib.pc_plan_sections(self._handle, None, 0, ctypes.byref(n)), "pc_plan_sections")
        arr = (SectionInfo * max(n.value, 1))()
        _check(self._lib, self._lib.pc_plan_sections(self._handle, arr, n.value, ctypes.byref(n)), "pc_plan_sections")
        return [{f: getattr(arr[i], f) for f, _ in SectionInfo._fields_} for i in range(n.value)]

    def apply_adjoint(self, v, out=None, stream=None):
        """``x = H_m^* v``."""
        v, out, batch = self._prep(v, out)
        st = self._lib.pc_apply_adjoint(self._handle, ctypes.c_void_p(v.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), batch,
                                        ctypes.c_void_p(_stream_ptr(stream, v.device)))
        _check(self._lib, st, "pc_apply_adjoint")
        return out

    def info(self) -> dict:
        inf = PlanInfo()
        _check(self._lib, self._lib.pc_plan_query(self._handle, ctypes.byref(inf)), "pc_plan_query")
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    @property
    def spectra_shape(self):
        """Shape of the natural-layout spectra: (m, N/2+1) or (m, N1, N2/2+1);
        for a sectioned plan the flat concatenation of its sections' spectra."""
        if getattr(self, "_spec_shape", None) is None:
            inf = self.info()
            if inf["path"] == 3:
                self._spec_shape = (int(inf["spectra_count"]),)
            else:
                self._spec_shape = (self.m,) + tuple(self.shape[:-1]) + (self.shape[-1] // 2 + 1,)
        return self._spec_shape

    def get_spectra(self, out=None, stream=None):
        """The operator's spectra as a complex64 CUDA tensor (real-FFT layout)."""
        import torch
        if out is None:
            out = torch.empty(self.spectra_shape, dtype=torch.complex64, device="cuda")
        self._check_spec(out)
        st = self._lib.pc_plan_get_spectra(self._handle, ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(_stream_ptr(stream, out.device)))
        _check(self._lib, st, "pc_plan_get_spectra")
        return out

    def set_spectra(self, spec, stream=None):
        """Replace the operator's spectra (complex64 CUDA tensor, real-FFT layout)."""
        spec = spec.contiguous()
        self._check_spec(spec)
        st = self._lib.pc_plan_set_spectra(self._handle, ctypes.c_void_p(spec.data_ptr()),
                                           ctypes.c_void_p(_stream_ptr(stream, spec.device)))
        _check(self._lib, st, "pc_plan_set_spectra")

    @classmethod
    def from_meyer(cls, n, levels, lowpass, lam, mu, c, batch=1, stream=None, gradients=False,
                   product_convolution=False):
        """Plan of Meyer's representation (section 4.5) from kept wavelet
        coefficients c[i] = c_{lam[i], mu[i]}; terms are the distinct mu in
        increasing order (see pc_plan_create_meyer)."""
        self = cls.__new__(cls)
        self._lib = load_library()
        self._handle = ctypes.c_void_p()
        lp = _f32(lowpass).ravel()
        lam = np.ascontiguousarray(np.asarray(lam, np.int64))
        mu = np.ascontiguousarray(np.asarray(mu, np.int64))
        c = _f32(c).ravel()
        if not (lam.shape == mu.shape == c.shape) or lam.ndim != 1:
            raise ValueError("lam, mu and c must be 1D of equal length")
        flags = (PC_PLAN_GRADIENTS if gradients else 0) | (PC_PLAN_PRODUCT_CONVOLUTION if product_convolution else 0)
        st = self._lib.pc_plan_create_meyer(ctypes.byref(self._handle), int(n), int(levels), lp.shape[0],
                                            lp.ctypes.data_as(ctypes.c_void_p), c.shape[0],
                                            lam.ctypes.data_as(ctypes.c_void_p), mu.ctypes.data_as(ctypes.c_void_p),
                                            c.ctypes.data_as(ctypes.c_void_p), int(batch), flags,
                                            ctypes.c_void_p(_stream_ptr(stream)))
        _check(self._lib, st, "pc_plan_create_meyer")
        self.m = int(np.unique(mu).shape[0])
        self.batch = int(batch)
        self.shape = (int(n),)
        self.product_convolution = bool(product_convolution)
        self.desc = None
        return self

    def set_responses(self, h, stream=None):
        """Replace the impulse responses by a float32 CUDA tensor (``m x N`` or
        ``m x N1 x N2``, lag layout); the spectra are recomputed on the device."""
        import torch
        if not (isinstance(h, torch.Tensor) and h.is_cuda and h.dtype == torch.float32):
            raise TypeError("h must be a float32 CUDA tensor")
        h = h.contiguous()
        if tuple(h.shape) != (self.m,) + self.shape:
            raise ValueError(f"h must be {(self.m,) + self.shape}, got {tuple(h.shape)}")
        self._h_keep = h  # alive until the enqueued transform has read it
        st = self._lib.pc_plan_set_responses(self._handle, ctypes.c_void_p(h.data_ptr()),
                                             ctypes.c_void_p(_stream_ptr(stream, h.device)))
        _check(self._lib, st, "pc_plan_set_responses")

    def grad_spectra(self, u, gy, out=None, stream=None):
        """dL/dspec given the forward input u and dL/dy (see pc_grad_spectra)."""
        import torch
        u, _, batch = self._prep(u, None)
        gy = gy.contiguous()
        if gy.shape != u.shape or gy.dtype != torch.float32 or not gy.is_cuda:
            raise ValueError("gy must be a float32 CUDA tensor shaped like u")
        if out is None:
            out = torch.empty(self.spectra_shape, dtype=torch.complex64, device=u.device)
        self._check_spec(out)
        st = self._lib.pc_grad_spectra(self._handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), batch,
                                       ctypes.c_void_p(_stream_ptr(stream, u.device)))
        _check(self._lib, st, "pc_grad_spectra")
        return out

    def _check_spec(self, t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex64 and t.is_contiguous()
                and tuple(t.shape) == self.spectra_shape):
            raise ValueError(f"spectra must be a contiguous complex64 CUDA tensor of shape {self.spectra_shape}")

    def set_tracing(self, enable: bool = True):
        """Bracket every kernel of later calls with HIP events (see pc.h)."""
        _check(self._lib, self._lib.pc_plan_set_tracing(self._handle, int(bool(enable))), "pc_plan_set_tracing")

    def trace_stats(self) -> dict:
        """Per-kernel {name: {launches, total_ms, min_ms, max_ms, avg_ms}} (waits for the events)."""
        cap = 32
        arr = (KernelStat * cap)()
        n = ctypes.c_int32()
        _check(self._lib, self._lib.pc_plan_trace_stats(self._handle, arr, cap, ctypes.byref(n)),
               "pc_plan_trace_stats")
        out = {}
        for i in range(min(n.value, cap)):
            r = arr[i]
            out[r.kernel.decode()] = {"launches": r.launches, "total_ms": r.total_ms, "min_ms": r.min_ms,
                                      "max_ms": r.max_ms,
                                      "avg_ms": r.total_ms / r.launches if r.launches else 0.0}
        return out

    def trace_reset(self):
        _check(self._lib, self._lib.pc_plan_trace_reset(self._handle), "pc_plan_trace_reset")

    def destroy(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            st = self._lib.pc_destroy(self._handle)
            self._handle = ctypes.c_void_p()
            _check(self._lib, st, "pc_destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def _lags_array(lags, n):
    lags = np.ascontiguousarray(np.asarray(lags, dtype=np.int64))
    if lags.ndim != 1:
        raise ValueError("lags must be one-dimensional")
    return lags


def construct_project(tvir, lags, windows, stream=None):
    """``h`` (``m x n``) of the L2 projection of the TVIR rows onto the span of
    the windows (section 4.2).  ``tvir``: float32 CUDA ``rows x n``;
    ``lags``: the rows' flat lag indices; ``windows``: float32 CUDA ``m x n``
    (2D grids flattened).  Synchronous."""
    import torch
    lib = load_library()
    tvir, windows = tvir.contiguous(), windows.contiguous()
    rows, n = tvir.shape
    m = windows.shape[0]
    lg = _lags_array(lags, n)
    if lg.shape[0] != rows or windows.shape[1] != n:
        raise ValueError("tvir, lags and windows disagree in size")
    h = torch.empty((m, n), dtype=torch.float32, device=tvir.device)
    st = lib.pc_construct_project(n, m, rows, ctypes.c_void_p(tvir.data_ptr()), lg.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.c_void_p(windows.data_ptr()), ctypes.c_void_p(h.data_ptr()),
                                  ctypes.c_void_p(_stream_ptr(stream, tvir.device)))
    _check(lib, st, "pc_construct_project")
    return h


def construct_interpolate(samples, lags, nodes, windows, stream=None):
    """``h`` (``m x n``) interpolating the TVIR samples at the nodes (section
    4.4).  ``samples``: float32 CUDA ``rows x m`` (T(lag r, node i));
    ``nodes``: m flat positions; ``windows``: float32 CUDA ``m x n``.
    Synchronous."""
    import torch
    lib = load_library()
    samples, windows = samples.contiguous(), windows.contiguous()
    rows, m = samples.shape
    n = windows.shape[1]
    lg = _lags_array(lags, n)
    nd = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64))
    if lg.shape[0] != rows or windows.shape[0] != m or nd.shape != (m,):
        raise ValueError("samples, lags, nodes and windows disagree in size")
    h = torch.empty((m, n), dtype=torch.float32, device=samples.device)
    st = lib.pc_construct_interpolate(n, m, rows, ctypes.c_void_p(samples.data_ptr()),
                                      lg.ctypes.data_as(ctypes.c_void_p), nd.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.c_void_p(windows.data_ptr()), ctypes.c_void_p(h.data_ptr()),
                                      ctypes.c_void_p(_stream_ptr(stream, samples.device)))
    _check(lib, st, "pc_construct_interpolate")
    return h


def wavelet_transform(x, lowpass, levels, inverse=False, axis=-1, stream=None, out=None, no_alloc=False):
    """Periodic orthonormal DWT (or its inverse) of a float32 CUDA tensor
    along ``axis`` (``x`` 1D, or 2D with axis 0 or 1), pyramid order.

    ``no_alloc=True`` calls ``pc_wavelet_transform_noalloc`` (fixed scratch,
    no device allocation, asynchronous; pass ``out`` to keep torch from
    allocating too)."""
    import torch
    lib = load_library()
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32) or x.dim() not in (1, 2):
        raise TypeError("x must be a 1D or 2D float32 CUDA tensor")
    x = x.contiguous()
    lp = _f32(lowpass).ravel()
    if x.dim() == 1:
        count, n, stride, dist = 1, x.shape[0], 1, x.shape[0]
    elif axis in (-1, 1):
        count, n, stride, dist = x.shape[0], x.shape[1], 1, x.shape[1]
    else:
        count, n, stride, dist = x.shape[1], x.shape[0], x.shape[1], 1
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor shaped like x")
    fn = lib.pc_wavelet_transform_noalloc if no_alloc else lib.pc_wavelet_transform
    st = fn(1 if inverse else 0, n, int(levels), lp.shape[0], lp.ctypes.data_as(ctypes.c_void_p),
            count, stride, dist, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(_stream_ptr(stream, x.device)))
    _check(lib, st, "pc_wavelet_transform_noalloc" if no_alloc else "pc_wavelet_transform")
    return out


class Batch:
    """Many 2D operators of uneven sizes run together (see pc_batch_create).

    ``plans``: distinct 2D :class:`Plan` objects (full-grid or sectioned).  ``apply(inputs)``
    enqueues ``H_i inputs[i]`` for every instance with one graph launch and
    returns the outputs (allocated here unless ``outputs`` is given);
    ``apply_adjoint`` the adjoints.  Each call may pass new tensors.  While
    the batch lives its plans cannot be destroyed.
    """

    def __init__(self, plans, graph: bool = True, persistent: bool = False, stream=None):
        self._lib = load_library()
        self.plans = list(plans)
        n = len(self.plans)
        self._handle = ctypes.c_void_p()
        hp = (ctypes.c_void_p * n)(*[p._handle.value for p in self.plans])
        flags = (0 if graph else PC_BATCH_NO_GRAPH) | (PC_BATCH_PERSISTENT if persistent else 0)
        st = self._lib.pc_batch_create(ctypes.byref(self._handle), n, hp, flags, ctypes.c_void_p(_stream_ptr(stream)))
        _check(self._lib, st, "pc_batch_create")

    def _call(self, fn, name, inputs, outputs, stream):
        import torch
        n = len(self.plans)
        inputs = [x.contiguous() for x in inputs]
        if len(inputs) != n:
            raise ValueError(f"{name}: {len(inputs)} inputs for {n} instances")
        outputs = [torch.empty_like(x) for x in inputs] if outputs is None else list(outputs)
        if len(outputs) != n or any(not y.is_contiguous() for y in outputs):
            raise ValueError(f"{name}: need {n} contiguous outputs")
        arr = lambda xs: (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])  # noqa: E731
        _check(self._lib, fn(self._handle, arr(inputs), arr(outputs), ctypes.c_void_p(_stream_ptr(stream))), name)
        return outputs

    def apply(self, inputs, outputs=None, stream=None):
        return self._call(self._lib.pc_batch_apply, "pc_batch_apply", inputs, outputs, stream)

    def apply_adjoint(self, inputs, outputs=None, stream=None):
        return self._call(self._lib.pc_batch_apply_adjoint, "pc_batch_apply_adjoint", inputs, outputs, stream)

    def destroy(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            st = self._lib.pc_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()
            _check(self._lib, st, "pc_batch_destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
