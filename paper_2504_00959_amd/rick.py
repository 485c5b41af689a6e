"""Python binding of the w-stacking imager's C ABI (``include/rick.h``).

Argument marshalling only: device tensors are passed as raw pointers with
the current HIP stream; every step of the imaging path runs in the HIP
kernels of ``librick.so``.  There is no fallback: if the library is missing
or fails, the call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RICK_LIB names another build of the same library (for instance one with
# host-side sanitizers); by default the one built next to this file
LIB_PATH = os.environ.get("RICK_LIB") or os.path.join(_HERE, "librick.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "rick.h")

RICK_OK = 0
STATUS_NAMES = {0: "RICK_OK", 1: "RICK_E_INVALID_ARG", 2: "RICK_E_NO_DEVICE", 3: "RICK_E_OOM", 4: "RICK_E_HIP",
                5: "RICK_E_CAPACITY", 6: "RICK_E_BAD_PLAN", 7: "RICK_E_STATE", 8: "RICK_E_UNSUPPORTED"}
KERNELS = {"gaussian": 0, "kaiser_bessel": 1, "kb": 1, "user_lut": 2}
MLP_PARAMS = 1217
PRECISIONS = {"fp32": 0, "fp32_kahan": 1, "fp64": 2}
FLAG_TIMING = 1
FLAG_FUSED_SCREEN = 2
FLAG_PLANE_ORIENT = 4


class RickError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({detail})")


class OrderInfo(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("panel", ctypes.c_int32), ("pad", ctypes.c_int32)]


class DegridOrder:
    """Sorted positions of one set of visibilities (rick_degrid_order_t)."""

    def __init__(self, handle, nrow: int, nchan: int, device: int = 0):
        self._h = handle
        self.nrow, self.nchan, self.device = nrow, nchan, device

    def arrays(self):
        """(keys, vals, panel): host uint64 copies of the order's sorted arrays
        (rick_degrid_order_info)."""
        import torch
        inf = OrderInfo()
        _check(lib().rick_degrid_order_info(self._h, ctypes.byref(inf)), "rick_degrid_order_info")
        out = []
        for ptr in (inf.keys, inf.vals):
            class _View:
                __cuda_array_interface__ = {"shape": (int(inf.n),), "typestr": "<i8", "data": (ptr, False),
                                            "version": 2, "strides": None}
            out.append(torch.as_tensor(_View(), device=f"cuda:{self.device}").cpu().numpy().view(np.uint64))
        return out[0], out[1], int(inf.panel)

    def close(self):
        if self._h:
            _check(lib().rick_degrid_order_destroy(self._h), "rick_degrid_order_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GridJob(ctypes.Structure):
    """rick_grid_job: one job of rick_grid_jobs."""
    _fields_ = [("plan", ctypes.c_void_p), ("uvw", ctypes.c_void_p), ("freq_hz", ctypes.POINTER(ctypes.c_double)),
                ("vis", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("nrow", ctypes.c_int64),
                ("nchan", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ImageJob(ctypes.Structure):
    """rick_image_job: one job of rick_wstack_image_jobs."""
    _fields_ = [("plan", ctypes.c_void_p), ("image", ctypes.c_void_p)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("grid_n", ctypes.c_int32), ("n_wplanes", ctypes.c_int32), ("support", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("kernel", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("kernel_param", ctypes.c_double), ("fov_rad", ctypes.c_double), ("w_min", ctypes.c_double),
                ("w_max", ctypes.c_double), ("max_vis", ctypes.c_int64), ("device", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("lut_wbins", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_gridded", ctypes.c_int64), ("n_dropped", ctypes.c_int64), ("n_records", ctypes.c_int64),
                ("sum_weights", ctypes.c_double), ("du", ctypes.c_double), ("dl", ctypes.c_double),
                ("dw", ctypes.c_double), ("mesh", ctypes.c_void_p), ("mesh_bytes", ctypes.c_int64),
                ("row_mesh", ctypes.c_void_p), ("panel", ctypes.c_int32), ("occ_words", ctypes.c_int32),
                ("tile_bits", ctypes.c_void_p), ("tiles_set", ctypes.c_int64), ("tile_rows_set", ctypes.c_int64),
                ("rec1_bytes", ctypes.c_int32), ("pad1", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32), ("state", ctypes.c_int32),
                ("n_timers", ctypes.c_int32), ("kernel_ms", ctypes.c_float * 16),
                ("kernel_calls", ctypes.c_int32 * 16), ("kernel_names", ctypes.c_char_p * 16),
                ("w_k", ctypes.POINTER(ctypes.c_double)), ("taper", ctypes.c_void_p), ("lut_wbins", ctypes.c_int32),
                ("pad2", ctypes.c_int32), ("plane_transposed", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librick.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the imager has no non-HIP path)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.rick_plan.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(P)]
    L.rick_grid.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), P, P, ctypes.c_int64, ctypes.c_int32, P]
    L.rick_grid_static.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), P, P, ctypes.c_int64, ctypes.c_int32, P]
    L.rick_grid_jobs.argtypes = [ctypes.POINTER(GridJob), ctypes.c_int32, P]
    L.rick_wstack_image_jobs.argtypes = [ctypes.POINTER(ImageJob), ctypes.c_int32, P]
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.rick_plan_set_lut.argtypes = [P, P, i32, P]
    L.rick_mlp_tabulate.argtypes = [P, i32, i32, i32, P, P]
    L.rick_mlp_backward.argtypes = [P, i32, i32, i32, P, P, P, P]
    L.rick_adam_step.argtypes = [P, P, P, P, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, P]
    L.rick_image_loss.argtypes = [P, P, P, P, P, P, P]
    L.rick_table_gradient.argtypes = [P, P, P, P, ctypes.POINTER(ctypes.c_double), P, P, i64, i32, P, P]
    L.rick_separable_table.argtypes = [P, i32, P, P]
    L.rick_table_residual.argtypes = [P, P, i64, P, P, P]
    L.rick_dft_image.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), P, P, i64, i32, i32, i32, i32, i32, P, P]
    L.rick_fft_planes.argtypes = [P, P]
    L.rick_wstack_image.argtypes = [P, P, P]
    L.rick_reset.argtypes = [P, P]
    L.rick_predict_planes.argtypes = [P, P, P]
    L.rick_degrid.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), P, ctypes.c_int64, ctypes.c_int32, P]
    L.rick_degrid_order_create.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int32,
                                           ctypes.POINTER(P), P]
    L.rick_degrid_sorted.argtypes = [P, P, P, P]
    L.rick_degrid_order_destroy.argtypes = [P]
    L.rick_degrid_order_info.argtypes = [P, ctypes.POINTER(OrderInfo)]
    L.rick_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    L.rick_plan_destroy.argtypes = [P]
    L.rick_plan_bin_counts.argtypes = [P, P, ctypes.c_int64]
    L.rick_plan_retarget.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.rick_capture_begin.argtypes = [P]
    L.rick_capture_end.argtypes = [P, ctypes.POINTER(P)]
    L.rick_graph_launch.argtypes = [P, P]
    L.rick_graph_destroy.argtypes = [P]
    L.rick_stamps_create.argtypes = [ctypes.c_int32, ctypes.POINTER(P)]
    L.rick_stamp.argtypes = [P, ctypes.c_int32, P]
    L.rick_stamps_elapsed.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]
    L.rick_stamps_destroy.argtypes = [P]
    L.rick_autotune.argtypes = [ctypes.POINTER(PlanDesc), P, ctypes.POINTER(ctypes.c_double), P, P, ctypes.c_int64,
                                ctypes.c_int32, P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_float)]
    for f in ("rick_plan_set_lut", "rick_mlp_tabulate", "rick_mlp_backward", "rick_adam_step", "rick_image_loss",
              "rick_table_gradient", "rick_dft_image", "rick_separable_table", "rick_table_residual",
              "rick_plan", "rick_grid", "rick_grid_static", "rick_grid_jobs", "rick_wstack_image_jobs", "rick_fft_planes", "rick_wstack_image", "rick_reset", "rick_plan_info",
              "rick_plan_destroy", "rick_plan_bin_counts", "rick_capture_begin", "rick_capture_end",
              "rick_graph_launch", "rick_graph_destroy", "rick_stamps_create", "rick_stamp", "rick_stamps_elapsed",
              "rick_stamps_destroy", "rick_autotune", "rick_plan_retarget", "rick_predict_planes", "rick_degrid",
              "rick_degrid_order_create", "rick_degrid_sorted", "rick_degrid_order_destroy",
              "rick_degrid_order_info"):
        getattr(L, f).restype = ctypes.c_int32
    L.rick_status_str.argtypes = [ctypes.c_int32]
    L.rick_status_str.restype = ctypes.c_char_p
    L.rick_last_error.argtypes = []
    L.rick_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def header_functions() -> list:
    """Names of the functions include/rick.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rick_\w+)\s*\(", txt, flags=re.M)


def _check(status: int, where: str):
    if status != RICK_OK:
        raise RickError(status, where, lib().rick_last_error().decode(errors="replace"))


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_desc(grid_n, n_wplanes, support, oversample, fov, w_min, w_max, kernel="gaussian", kernel_param=0.0,
              precision="fp32", max_vis=1 << 20, device=0, timing=False, tile=0, chunk=0,
              fused=False, lut_wbins=0, orient=False) -> PlanDesc:
    flags = (FLAG_TIMING if timing else 0) | (FLAG_FUSED_SCREEN if fused else 0) | (FLAG_PLANE_ORIENT if orient else 0)
    return PlanDesc(grid_n=grid_n, n_wplanes=n_wplanes, support=support, oversample=oversample,
                    kernel=KERNELS[kernel], precision=PRECISIONS[precision], kernel_param=kernel_param,
                    fov_rad=fov, w_min=w_min, w_max=w_max, max_vis=max_vis, device=device,
                    flags=flags, tile=tile, chunk=chunk, lut_wbins=lut_wbins)


class Plan:
    """One imaging plan (device buffers allocated once at construction)."""

    def __init__(self, grid_n: int, n_wplanes: int, support: int, oversample: int, fov: float, w_min: float,
                 w_max: float, kernel: str = "gaussian", kernel_param: float = 0.0, precision: str = "fp32",
                 max_vis: int = 1 << 20, device: int = 0, timing: bool = False, tile: int = 0, chunk: int = 0,
                 fused: bool = False, lut_wbins: int = 0, orient: bool = False):
        self.desc = make_desc(grid_n, n_wplanes, support, oversample, fov, w_min, w_max, kernel, kernel_param,
                              precision, max_vis, device, timing, tile, chunk, fused, lut_wbins, orient)
        self.support, self.oversample, self.lut_wbins = support, oversample, lut_wbins
        self.fused = fused
        self.precision = precision
        self.grid_n = grid_n
        self.n_wplanes = n_wplanes
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().rick_plan(ctypes.byref(self.desc), ctypes.byref(h)), "rick_plan")
        self._h = h

    @classmethod
    def for_dataset(cls, ds, **kw):
        args = dict(ds.plan_kwargs())
        args.setdefault("max_vis", max(1, ds.nvis))
        args.update(kw)
        return cls(**args)

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    def _device_tensor(self, t, name, dtype):
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda" or (t.device.index or 0) != self.device:
            raise ValueError(f"{name} must be on cuda:{self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def grid(self, uvw, vis, weight=None, freq: Optional[Sequence[float]] = None, stream=None,
             static_scratch: bool = False):
        """Bin-and-sort + grid.  uvw float64 [R,3] (metres if freq given, else wavelengths),
        vis complex [R,C], weight float32 [R,C] or None, freq host sequence [C] in Hz or None.
        static_scratch: call rick_grid_static (sort buffers in the library's static
        device scratch; nothing allocated) instead of rick_grid."""
        a = self._grid_args(uvw, vis, weight, freq)
        fn, name = (lib().rick_grid_static, "rick_grid_static") if static_scratch else (lib().rick_grid, "rick_grid")
        _check(fn(self._h, a.uvw, a.freq_hz, a.vis, a.weight, a.nrow, a.nchan, _stream_handle(stream)), name)

    def _grid_args(self, uvw, vis, weight, freq) -> "GridJob":
        """Checked arguments of one rick_grid call as a rick_grid_job (the
        frequency array is kept alive by the plan until its next call)."""
        import torch
        self._device_tensor(uvw, "uvw", torch.float64)
        self._device_tensor(vis, "vis", self.complex_dtype)
        if uvw.dim() != 2 or uvw.shape[1] != 3:
            raise ValueError("uvw must be [nrow, 3]")
        nrow = uvw.shape[0]
        if vis.dim() == 1:
            vis = vis.reshape(nrow, 1)
        nchan = vis.shape[1]
        if vis.shape[0] != nrow:
            raise ValueError("vis must be [nrow, nchan]")
        wptr = None
        if weight is not None:
            self._device_tensor(weight, "weight", torch.float32)
            if weight.numel() != nrow * nchan:
                raise ValueError("weight must be [nrow, nchan]")
            wptr = weight.data_ptr()
        fptr = None
        if freq is not None:
            f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).reshape(-1))
            if f.shape[0] != nchan:
                raise ValueError("freq must have nchan entries")
            self._freq_keep = f
            fptr = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return GridJob(self._h, uvw.data_ptr(), fptr, vis.data_ptr(), wptr, nrow, nchan, 0)

    def fft(self, stream=None):
        _check(lib().rick_fft_planes(self._h, _stream_handle(stream)), "rick_fft_planes")

    def image(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.grid_n, self.grid_n), dtype=self.real_dtype, device=f"cuda:{self.device}")
        self._device_tensor(out, "out", self.real_dtype)
        if out.numel() != self.grid_n * self.grid_n:
            raise ValueError("out must be [N, N]")
        _check(lib().rick_wstack_image(self._h, out.data_ptr(), _stream_handle(stream)), "rick_wstack_image")
        return out

    def predict_planes(self, model, stream=None):
        """Prediction, first half: the model image (device [N, N], the plan's
        real dtype) to the planes' forward transforms (held conjugated)."""
        self._device_tensor(model, "model", self.real_dtype)
        if model.numel() != self.grid_n * self.grid_n:
            raise ValueError("model must be [N, N]")
        _check(lib().rick_predict_planes(self._h, model.data_ptr(), _stream_handle(stream)), "rick_predict_planes")

    def degrid(self, uvw, freq: Optional[Sequence[float]] = None, out=None, stream=None):
        """Prediction, second half: visibilities [nrow, nchan] (complex, the
        plan's precision) at uvw (float64 [nrow, 3], metres if freq is given,
        else wavelengths) from the predicted planes."""
        import torch
        self._device_tensor(uvw, "uvw", torch.float64)
        if uvw.dim() != 2 or uvw.shape[1] != 3:
            raise ValueError("uvw must be [nrow, 3]")
        nrow = uvw.shape[0]
        fptr = None
        nchan = 1
        if freq is not None:
            f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).reshape(-1))
            nchan = f.shape[0]
            self._freq_keep = f
            fptr = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if out is None:
            out = torch.empty((nrow, nchan), dtype=self.complex_dtype, device=f"cuda:{self.device}")
        self._device_tensor(out, "out", self.complex_dtype)
        if out.numel() != nrow * nchan:
            raise ValueError("out must be [nrow, nchan]")
        _check(lib().rick_degrid(self._h, uvw.data_ptr(), fptr, out.data_ptr(), nrow, nchan, _stream_handle(stream)),
               "rick_degrid")
        return out

    def degrid_order(self, uvw, freq: Optional[Sequence[float]] = None, stream=None) -> "DegridOrder":
        """Quantise and sort the positions once for repeated prediction
        (valid for this plan's current grid, field and w range)."""
        import torch
        self._device_tensor(uvw, "uvw", torch.float64)
        if uvw.dim() != 2 or uvw.shape[1] != 3:
            raise ValueError("uvw must be [nrow, 3]")
        nrow = uvw.shape[0]
        fptr, nchan, f = None, 1, None
        if freq is not None:
            f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).reshape(-1))
            nchan = f.shape[0]
            fptr = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(lib().rick_degrid_order_create(self._h, uvw.data_ptr(), fptr, nrow, nchan, ctypes.byref(h),
                                              _stream_handle(stream)), "rick_degrid_order_create")
        return DegridOrder(h, nrow, nchan, self.device)

    def degrid_sorted(self, order: "DegridOrder", out=None, stream=None):
        """rick_degrid over a sort order's visibilities; returns [nrow, nchan]."""
        import torch
        if out is None:
            out = torch.empty((order.nrow, order.nchan), dtype=self.complex_dtype, device=f"cuda:{self.device}")
        self._device_tensor(out, "out", self.complex_dtype)
        if out.numel() != order.nrow * order.nchan:
            raise ValueError("out must be [nrow, nchan]")
        _check(lib().rick_degrid_sorted(self._h, order._h, out.data_ptr(), _stream_handle(stream)),
               "rick_degrid_sorted")
        return out

    # ---- learned gridding kernel ----
    def set_lut(self, table, stream=None):
        """Install a table [N_f, OS, OS, W, W] (float32: device tensor, or host
        numpy array) into a user-table plan and compute its taper."""
        import torch
        if isinstance(table, torch.Tensor):
            self._device_tensor(table, "table", torch.float32)
            _check(lib().rick_plan_set_lut(self._h, table.data_ptr(), 1, _stream_handle(stream)), "rick_plan_set_lut")
        else:
            t = np.ascontiguousarray(np.asarray(table, dtype=np.float32))
            _check(lib().rick_plan_set_lut(self._h, t.ctypes.data, 0, _stream_handle(stream)), "rick_plan_set_lut")

    def separable_table(self, n_wbins: int, out=None, stream=None):
        """rick_separable_table: this (Gaussian or Kaiser-Bessel) plan's taps as a
        user table [n_wbins, OS, OS, W, W] (float32, device)."""
        import torch
        shape = (n_wbins, self.oversample, self.oversample, self.support, self.support)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=f"cuda:{self.device}")
        self._device_tensor(out, "out", torch.float32)
        if tuple(out.shape) != shape:
            raise ValueError("out has the wrong shape")
        _check(lib().rick_separable_table(self._h, n_wbins, out.data_ptr(), _stream_handle(stream)),
               "rick_separable_table")
        return out

    def taper(self):
        """Device float64 view of the taper the image is divided by: [N] (separable) or [N, N] (user table)."""
        inf = self.info()
        shape = (self.grid_n, self.grid_n) if inf["lut_wbins"] else (self.grid_n,)
        return self._device_view(inf["taper_ptr"], shape, "<f8")

    def image_loss(self, image, target, dimage, dtaper, sums, stream=None):
        """rick_image_loss: sums[0] / sums[1] is the loss; dimage, dtaper its gradients (float64 [N, N])."""
        import torch
        self._device_tensor(image, "image", self.real_dtype)
        for t, n in ((target, "target"), (dimage, "dimage"), (dtaper, "dtaper")):
            self._device_tensor(t, n, torch.float64)
            if t.numel() != self.grid_n * self.grid_n:
                raise ValueError(f"{n} must be [N, N]")
        self._device_tensor(sums, "sums", torch.float64)
        if sums.numel() < 2:
            raise ValueError("sums must hold 2 values")
        _check(lib().rick_image_loss(self._h, image.data_ptr(), target.data_ptr(), dimage.data_ptr(),
                                     dtaper.data_ptr(), sums.data_ptr(), _stream_handle(stream)), "rick_image_loss")

    def table_gradient(self, dimage, dtaper, uvw, vis, weight, freq, dtable, stream=None):
        """rick_table_gradient: dL/dT (float64 [N_f, OS, OS, W, W]) for the visibilities just imaged."""
        import torch
        self._device_tensor(dimage, "dimage", torch.float64)
        self._device_tensor(dtaper, "dtaper", torch.float64)
        self._device_tensor(dtable, "dtable", torch.float64)
        self._device_tensor(uvw, "uvw", torch.float64)
        self._device_tensor(vis, "vis", self.complex_dtype)
        nrow = uvw.shape[0]
        nchan = vis.numel() // max(1, nrow)
        if dtable.numel() != self.lut_wbins * self.oversample ** 2 * self.support ** 2:
            raise ValueError("dtable has the wrong size")
        wptr = None
        if weight is not None:
            self._device_tensor(weight, "weight", torch.float32)
            wptr = weight.data_ptr()
        fptr, f = None, None
        if freq is not None:
            f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).reshape(-1))
            fptr = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(lib().rick_table_gradient(self._h, dimage.data_ptr(), dtaper.data_ptr(), uvw.data_ptr(), fptr,
                                         vis.data_ptr(), wptr, nrow, nchan, dtable.data_ptr(),
                                         _stream_handle(stream)), "rick_table_gradient")

    def dft_image(self, uvw, vis, weight=None, freq=None, q0=0, p0=0, nq=None, np_=None, out=None, stream=None):
        """rick_dft_image: the direct Fourier sum at pixels [q0, q0 + nq) x [p0, p0 + np) (float64)."""
        import torch
        nq = self.grid_n if nq is None else nq
        np_ = self.grid_n if np_ is None else np_
        self._device_tensor(uvw, "uvw", torch.float64)
        self._device_tensor(vis, "vis", self.complex_dtype)
        nrow = uvw.shape[0]
        nchan = vis.numel() // max(1, nrow)
        wptr = None
        if weight is not None:
            self._device_tensor(weight, "weight", torch.float32)
            wptr = weight.data_ptr()
        fptr, f = None, None
        if freq is not None:
            f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).reshape(-1))
            fptr = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if out is None:
            out = torch.empty((nq, np_), dtype=torch.float64, device=f"cuda:{self.device}")
        self._device_tensor(out, "out", torch.float64)
        _check(lib().rick_dft_image(self._h, uvw.data_ptr(), fptr, vis.data_ptr(), wptr, nrow, nchan, q0, p0, nq, np_,
                                    out.data_ptr(), _stream_handle(stream)), "rick_dft_image")
        return out

    def retarget(self, fov: float, w_min: float, w_max: float):
        """Field of view and w range for the work issued next (host-side only)."""
        _check(lib().rick_plan_retarget(self._h, fov, w_min, w_max), "rick_plan_retarget")

    def reset(self, stream=None):
        _check(lib().rick_reset(self._h, _stream_handle(stream)), "rick_reset")

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().rick_plan_info(self._h, ctypes.byref(inf)), "rick_plan_info")
        timers = {}
        for i in range(inf.n_timers):
            name = inf.kernel_names[i]
            if name:
                timers[name.decode()] = (float(inf.kernel_ms[i]), int(inf.kernel_calls[i]))
        return dict(n_gridded=inf.n_gridded, n_dropped=inf.n_dropped, n_records=inf.n_records,
                    sum_weights=inf.sum_weights, du=inf.du, dl=inf.dl, dw=inf.dw, mesh_ptr=inf.mesh,
                    mesh_bytes=inf.mesh_bytes, row_mesh_ptr=inf.row_mesh, panel=inf.panel,
                    tile_bits_ptr=inf.tile_bits, occ_words=inf.occ_words, tiles_set=inf.tiles_set,
                    tile_rows_set=inf.tile_rows_set, rec1_bytes=inf.rec1_bytes, tile=inf.tile,
                    chunk=inf.chunk, state=inf.state, timers=timers,
                    w_k=np.array([inf.w_k[k] for k in range(self.n_wplanes)]), taper_ptr=inf.taper,
                    lut_wbins=inf.lut_wbins, plane_transposed_ptr=inf.plane_transposed)

    def bin_counts(self, n_bins: int) -> np.ndarray:
        """Per-(plane, tile) record counts of the last grid() (host int32 array)."""
        out = np.zeros(n_bins, dtype=np.int32)
        _check(lib().rick_plan_bin_counts(self._h, out.ctypes.data, n_bins), "rick_plan_bin_counts")
        return out

    def _device_view(self, ptr, shape, typestr=None):
        import torch
        ts = typestr or ("<c16" if self.precision == "fp64" else "<c8")

        class _View:
            __cuda_array_interface__ = {"shape": shape, "typestr": ts, "data": (ptr, False), "version": 2,
                                        "strides": None}
        return torch.as_tensor(_View(), device=f"cuda:{self.device}")

    def transposed(self) -> np.ndarray:
        """Host bool [N_w]: planes stored transposed (all False without orient)."""
        inf = self.info()
        if not inf["plane_transposed_ptr"]:
            return np.zeros(self.n_wplanes, dtype=bool)
        return self._device_view(inf["plane_transposed_ptr"], (self.n_wplanes,), "<i4").cpu().numpy() != 0

    def _stored_tile_mask(self):
        inf = self.info()
        nt, ow = self.grid_n // inf["tile"], inf["occ_words"]
        words = self._device_view(inf["tile_bits_ptr"], (self.n_wplanes * nt * ow,), "<i8")
        w = words.cpu().numpy().view(np.uint64).reshape(self.n_wplanes, nt, ow)
        bits = (w[..., :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
        return bits.reshape(self.n_wplanes, nt, ow * 64)[..., :nt].astype(bool)

    def tile_mask(self):
        """Host bool array [N_w, nt, nt]: tiles gridded onto since the last
        reset, as (plane, tile row, tile column) of G_k."""
        t = self._stored_tile_mask()
        tr = self.transposed()
        t[tr] = np.transpose(t[tr], (0, 2, 1))
        return t

    def _cell_mask(self, rows_only=False):
        """Device bool [N_w, N, N] of the cells the stored planes hold
        (tile-row granularity with rows_only)."""
        import torch
        t = self._stored_tile_mask()
        if rows_only:
            t = np.repeat(t.any(axis=2, keepdims=True), t.shape[2], axis=2)
        T = self.grid_n // t.shape[1]
        m = torch.as_tensor(t, device=f"cuda:{self.device}")
        return m.repeat_interleave(T, dim=1).repeat_interleave(T, dim=2)

    def mesh(self):
        """Copy of the planes: G_k after grid() (tiles not gridded onto since
        the reset read as zeros), F_k after fft() (G_k with the fused screen);
        complex [N_w, N, N] on the device."""
        inf = self.info()
        v = self._device_view(inf["mesh_ptr"], (self.n_wplanes, self.grid_n, self.grid_n)).clone()
        if inf["state"] == 1 or (inf["state"] == 2 and self.fused):
            v[~self._cell_mask()] = 0
            tr = self.transposed()
            if tr.any():          # planes stored transposed, back to G_k
                idx = np.nonzero(tr)[0]
                v[idx] = v[idx].transpose(1, 2).contiguous()
        return v

    def row_mesh(self):
        """With the fused screen, copy of the row transforms H_k written by fft(),
        reordered from column panels to [N_w, N, N] (row-major; rows of empty
        tile rows read as zeros; a plane stored transposed holds the row
        transforms of G_k^T); None otherwise."""
        inf = self.info()
        if not inf["row_mesh_ptr"]:
            return None
        pw, n = inf["panel"], self.grid_n
        v = self._device_view(inf["row_mesh_ptr"], (self.n_wplanes, n // pw, n, pw))
        v = v.permute(0, 2, 1, 3).reshape(self.n_wplanes, n, n).clone()
        v[~self._cell_mask(rows_only=True)] = 0
        return v

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().rick_plan_destroy(self._h), "rick_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def mlp_tabulate(theta, support: int, oversample: int, n_wbins: int, out=None, stream=None):
    """rick_mlp_tabulate: table [N_f, OS, OS, W, W] (float32, device) of the MLP parameters theta."""
    import torch
    if not (isinstance(theta, torch.Tensor) and theta.is_cuda and theta.dtype == torch.float32
            and theta.is_contiguous() and theta.numel() == MLP_PARAMS):
        raise TypeError(f"theta must be a contiguous float32 device tensor of {MLP_PARAMS}")
    shape = (n_wbins, oversample, oversample, support, support)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=theta.device)
    if out.dtype != torch.float32 or not out.is_contiguous() or tuple(out.shape) != shape:
        raise ValueError("out must be a contiguous float32 tensor of the table's shape")
    _check(lib().rick_mlp_tabulate(theta.data_ptr(), support, oversample, n_wbins, out.data_ptr(),
                                   _stream_handle(stream)), "rick_mlp_tabulate")
    return out


def mlp_backward(theta, table, dtable, dtheta=None, stream=None):
    """rick_mlp_backward: gradient of sum(dtable * table) with respect to theta (float32, device)."""
    import torch
    n_wbins, os_, _, w, _ = table.shape
    if dtable.dtype != torch.float64 or tuple(dtable.shape) != tuple(table.shape) or not dtable.is_contiguous():
        raise ValueError("dtable must be a contiguous float64 tensor of the table's shape")
    if dtheta is None:
        dtheta = torch.empty(MLP_PARAMS, dtype=torch.float32, device=theta.device)
    _check(lib().rick_mlp_backward(theta.data_ptr(), w, os_, n_wbins, table.data_ptr(), dtable.data_ptr(),
                                   dtheta.data_ptr(), _stream_handle(stream)), "rick_mlp_backward")
    return dtheta


def table_residual(table, target, dtable, sums, stream=None):
    """rick_table_residual: dtable = 2 (table - target) / n, sums[0] = mean squared difference."""
    n = table.numel()
    if target.numel() != n or dtable.numel() != n or sums.numel() < 1:
        raise ValueError("sizes do not match")
    _check(lib().rick_table_residual(table.data_ptr(), target.data_ptr(), n, dtable.data_ptr(), sums.data_ptr(),
                                     _stream_handle(stream)), "rick_table_residual")


def grid_jobs(jobs, stream=None):
    """rick_grid_jobs: each job (plan, uvw, vis[, weight[, freq]]) binned on
    its own plan, then the gridding of all jobs in one persistent launch per
    (support, tile edge).  Same argument rules as Plan.grid."""
    jobs = list(jobs)
    if not jobs:
        raise ValueError("no jobs")
    arr = (GridJob * len(jobs))()
    for i, job in enumerate(jobs):
        plan, uvw, vis = job[0], job[1], job[2]
        weight = job[3] if len(job) > 3 else None
        freq = job[4] if len(job) > 4 else None
        arr[i] = plan._grid_args(uvw, vis, weight, freq)
    _check(lib().rick_grid_jobs(arr, len(jobs), _stream_handle(stream)), "rick_grid_jobs")


def wstack_image_jobs(jobs, stream=None):
    """rick_wstack_image_jobs: each job (plan, image) -- image a contiguous
    device tensor [N, N] of the plan's real dtype -- as Plan.image would
    write it, the fused column passes of one grid size in one launch."""
    jobs = list(jobs)
    if not jobs:
        raise ValueError("no jobs")
    arr = (ImageJob * len(jobs))()
    for i, (plan, img) in enumerate(jobs):
        plan._device_tensor(img, "image", plan.real_dtype)
        if tuple(img.shape) != (plan.grid_n, plan.grid_n):
            raise ValueError("image must be [grid_n, grid_n]")
        arr[i] = ImageJob(plan._h, img.data_ptr())
    _check(lib().rick_wstack_image_jobs(arr, len(jobs), _stream_handle(stream)), "rick_wstack_image_jobs")


def adam_step(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """rick_adam_step on float32 device tensors of equal size."""
    n = theta.numel()
    for t in (grad, m, v):
        if t.numel() != n or not t.is_contiguous():
            raise ValueError("Adam buffers must match theta")
    _check(lib().rick_adam_step(theta.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), n, step, lr, beta1,
                                beta2, eps, _stream_handle(stream)), "rick_adam_step")


class Graph:
    """Work recorded from a stream (``rick_capture_begin`` / ``rick_capture_end``)
    and replayed with ``launch``.  Use ``with Graph.record(stream) as g:`` and
    issue the plan calls on that stream inside the block."""

    def __init__(self):
        self._h = None

    @classmethod
    def record(cls, stream=None):
        return _Recording(cls(), stream)

    def launch(self, stream=None):
        _check(lib().rick_graph_launch(self._h, _stream_handle(stream)), "rick_graph_launch")

    def close(self):
        if self._h:
            _check(lib().rick_graph_destroy(self._h), "rick_graph_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Recording:
    def __init__(self, graph, stream):
        self.graph, self.stream = graph, stream

    def __enter__(self):
        _check(lib().rick_capture_begin(_stream_handle(self.stream)), "rick_capture_begin")
        return self.graph

    def __exit__(self, exc_type, *a):
        h = ctypes.c_void_p()
        st = lib().rick_capture_end(_stream_handle(self.stream), ctypes.byref(h))
        if exc_type is None:
            _check(st, "rick_capture_end")
            self.graph._h = h
        elif st == RICK_OK:
            lib().rick_graph_destroy(h)


class Stamps:
    """Device timestamp slots (``rick_stamp`` may be recorded into a graph)."""

    def __init__(self, n: int):
        h = ctypes.c_void_p()
        _check(lib().rick_stamps_create(n, ctypes.byref(h)), "rick_stamps_create")
        self._h, self.n = h, n

    def stamp(self, i: int, stream=None):
        _check(lib().rick_stamp(self._h, i, _stream_handle(stream)), "rick_stamp")

    def elapsed(self, i: int, j: int) -> float:
        ms = ctypes.c_float()
        _check(lib().rick_stamps_elapsed(self._h, i, j, ctypes.byref(ms)), "rick_stamps_elapsed")
        return float(ms.value)

    def close(self):
        if self._h:
            _check(lib().rick_stamps_destroy(self._h), "rick_stamps_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ds, uvw, vis, weight=None, precision="fp32", device=0, fused=True, stream=None, orient=False):
    """Fastest (tile, chunk) for a job, by ``rick_autotune``; returns (tile, chunk, ms)."""
    args = dict(ds.plan_kwargs())
    args.setdefault("max_vis", max(1, ds.nvis))
    desc = make_desc(precision=precision, device=device, fused=fused, orient=orient, **args)
    nrow = int(uvw.shape[0])
    nchan = 1 if ds.freq is None else len(ds.freq)
    freq = None if ds.freq is None else (ctypes.c_double * nchan)(*[float(f) for f in ds.freq])
    t, c, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    _check(lib().rick_autotune(ctypes.byref(desc), uvw.data_ptr(), freq, vis.data_ptr(),
                               None if weight is None else weight.data_ptr(), nrow, nchan, _stream_handle(stream),
                               ctypes.byref(t), ctypes.byref(c), ctypes.byref(ms)), "rick_autotune")
    return int(t.value), int(c.value), float(ms.value)


def wstack_image(ds, device: int = 0, precision: str = "fp32", **kw):
    """Convenience: reset + grid + fft + image for a synth.Dataset whose arrays
    are moved to the device; returns (image tensor, plan info)."""
    import torch
    dev = f"cuda:{device}"
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to(dev)
    cd = torch.complex128 if precision == "fp64" else torch.complex64
    vis = ds.vis if isinstance(ds.vis, torch.Tensor) else torch.as_tensor(ds.vis)
    vis = vis.to(device=dev, dtype=cd).contiguous()
    wt = None if ds.weight is None else torch.as_tensor(ds.weight, dtype=torch.float32).to(dev).contiguous()
    with Plan.for_dataset(ds, precision=precision, device=device, **kw) as p:
        p.reset()
        p.grid(uvw, vis, wt, ds.freq)
        p.fft()
        img = p.image()
        torch.cuda.synchronize(dev)
        return img, p.info()
