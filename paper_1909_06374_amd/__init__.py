"""MI355X (gfx950) light-curve generator: Python binding of ``libagn.so``.

The functions below carry the names of the C ABI in ``include/agn.h`` and
only marshal arguments: every step of the method runs in the HIP kernels of
the library.  Tensors are torch tensors on the GPU (PyTorch supplies device
memory and streams); ``stream=None`` means the current torch stream.

Importing this package never falls back to another implementation: if the
library is not built, every call raises.
"""
from __future__ import annotations

import ctypes as C
import functools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagn.so")

AGN_FP64 = 0
AGN_FP32 = 1
AGN_OK = 0
AGN_EINVAL = -1
AGN_EUNSUPPORTED_N = -2
AGN_ENOMEM = -3
AGN_EDEVICE = -4

_lib = None


class AgnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"agn error {code}: {msg}")
        self.code = code


class agn_psd_params(C.Structure):
    """Eq. 3 parameters: norm (<= 0: unit variance), f_br, a_low, a_high."""
    _fields_ = [("norm", C.c_double), ("f_br", C.c_double),
                ("a_low", C.c_double), ("a_high", C.c_double)]


def psd_params(norm=0.0, f_br=1.0, a_low=1.0, a_high=2.0):
    return agn_psd_params(float(norm), float(f_br), float(a_low), float(a_high))


class agn_erdf_params(C.Structure):
    """Broken power law in dN/dlog10(lambda): u_min, u_max, u_br, d1, d2."""
    _fields_ = [("u_min", C.c_double), ("u_max", C.c_double), ("u_br", C.c_double),
                ("d1", C.c_double), ("d2", C.c_double)]


def erdf_params(u_min=-4.0, u_max=0.0, u_br=-1.5, d1=0.4, d2=2.5):
    return agn_erdf_params(float(u_min), float(u_max), float(u_br), float(d1), float(d2))


AGN_PDF_SHARP_BPL, AGN_PDF_EQ1, AGN_PDF_LOGNORMAL = 0, 1, 2
AGN_PDF_PER_LOG, AGN_PDF_PER_LINEAR = 0, 1


class agn_pdf_params(C.Structure):
    """General PDF in u = log10(lambda): kind (sharp BPL / Eq. 1 / Eq. 2), measure
    (dN/dlog10 lambda or dN/dlambda), u_min, u_max, u_star, d1, d2, sigma."""
    _fields_ = [("kind", C.c_int32), ("measure", C.c_int32), ("u_min", C.c_double),
                ("u_max", C.c_double), ("u_star", C.c_double), ("d1", C.c_double),
                ("d2", C.c_double), ("sigma", C.c_double)]


def pdf_params(kind, measure=AGN_PDF_PER_LOG, u_min=-3.75, u_max=0.5, u_star=-0.958607314841775, d1=0.47,
               d2=2.53, sigma=0.64):
    """Defaults: the Eq. 1 parameters of the reference simulation (Table 2:
    lambda* = 0.11, slopes 0.47 / 2.53, log lambda in [-3.75, 0.5])."""
    return agn_pdf_params(int(kind), int(measure), float(u_min), float(u_max), float(u_star), float(d1),
                          float(d2), float(sigma))


def _declare(lib):
    i32, i64, u32, u64, d = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    vp, sz = C.c_void_p, C.c_size_t
    pp = C.POINTER(agn_psd_params)
    lib.agn_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    lib.agn_ctx_destroy.argtypes = [vp]
    lib.agn_last_error.argtypes = []
    lib.agn_last_error.restype = C.c_char_p
    lib.agn_supported_n.argtypes = [i64]
    lib.agn_spectrum_workspace_size.argtypes = [i64, C.POINTER(sz)]
    lib.agn_workspace_size.argtypes = [i64, C.c_int, C.POINTER(sz)]
    lib.agn_batch_workspace_size.argtypes = [i32, vp, C.c_int, C.POINTER(sz)]
    lib.agn_psd_spectrum.argtypes = [vp, pp, i64, d, u64, u32, C.c_int, vp, vp, sz, vp]
    lib.agn_psd_spectrum_noalloc.argtypes = [vp, pp, i64, d, u64, u32, C.c_int, vp, vp]
    lib.agn_lc_iterate.argtypes = [vp, vp, vp, i64, i32, d, C.c_int, vp, vp, vp, vp, vp, sz, vp]
    lib.agn_lc_generate.argtypes = [vp, pp, vp, i64, d, i32, d, u64, u32, C.c_int, vp, vp, vp,
                                    vp, sz, vp]
    lib.agn_lc_generate_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, d, C.c_int,
                                          vp, vp, vp, vp, sz, vp]
    lib.agn_test_philox.argtypes = [u64, u64, u64, i64, vp, vp]
    lib.agn_test_workspace_size.argtypes = [i64, C.c_int, i32, C.POINTER(sz)]
    lib.agn_test_lds_bandwidth.argtypes = [i32, i32, vp, C.POINTER(d), vp]
    for f in ("agn_test_rfft", "agn_test_irfft", "agn_test_argsort"):
        getattr(lib, f).argtypes = [vp, vp, i64, C.c_int, i32, vp, vp, sz, vp]
    lib.agn_erdf_draw.argtypes = [vp, C.POINTER(agn_erdf_params), i64, u64, u32, vp, vp]
    lib.agn_pdf_draw.argtypes = [vp, C.POINTER(agn_pdf_params), i64, u64, u32, vp, vp]
    lib.agn_lag_stats_workspace_size.argtypes = [i32, vp, i32, vp, i32, i32, C.POINTER(sz)]
    lib.agn_lag_stats_batch.argtypes = [vp, i32, vp, vp, vp, i32, vp, i32, vp, vp, i32, vp, d, vp, vp, vp, sz, vp]
    lib.agn_psd_fit_workspace_size.argtypes = [i32, vp, d, C.POINTER(sz)]
    lib.agn_psd_fit_batch.argtypes = [vp, i32, vp, vp, vp, d, vp, vp, vp, vp, sz, vp]
    lib.agn_pdf_slice.argtypes = [vp, C.POINTER(agn_pdf_params), i64, i32, i32, u64, u32, vp, vp]
    lib.agn_batch_plan_create.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, d, C.c_int, vp, vp, vp,
                                          C.c_int, C.c_int, vp, sz, vp, C.POINTER(vp)]
    lib.agn_batch_plan_launch.argtypes = [vp, vp]
    lib.agn_batch_plan_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.agn_batch_plan_tuning.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.agn_batch_plan_destroy.argtypes = [vp]
    lib.agn_log_bin_count.argtypes = [i64, d, C.POINTER(i32)]
    lib.agn_periodogram_workspace_size.argtypes = [i32, vp, d, C.POINTER(sz)]
    lib.agn_periodogram_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, d, vp, vp, vp, sz, vp]
    lib.agn_ctx_set_profiling.argtypes = [vp, C.c_int]
    lib.agn_ctx_set_lookback_polls.argtypes = [vp, i32]
    lib.agn_ctx_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(d), C.POINTER(i64), C.c_int]
    lib.agn_ctx_kernel_names.argtypes = []
    lib.agn_ctx_kernel_names.restype = C.c_char_p
    for f in ("agn_ctx_create", "agn_ctx_destroy", "agn_supported_n", "agn_spectrum_workspace_size",
              "agn_workspace_size", "agn_batch_workspace_size", "agn_psd_spectrum", "agn_psd_spectrum_noalloc",
              "agn_lc_iterate", "agn_lc_generate", "agn_lc_generate_batch", "agn_test_philox",
              "agn_ctx_set_profiling", "agn_ctx_set_lookback_polls", "agn_ctx_kernel_time", "agn_erdf_draw", "agn_pdf_draw", "agn_pdf_slice", "agn_batch_plan_create",
              "agn_batch_plan_launch", "agn_batch_plan_info", "agn_batch_plan_tuning", "agn_batch_plan_destroy", "agn_log_bin_count",
              "agn_periodogram_workspace_size", "agn_periodogram_batch", "agn_lag_stats_workspace_size",
              "agn_lag_stats_batch", "agn_psd_fit_workspace_size", "agn_psd_fit_batch",
              "agn_test_workspace_size", "agn_test_rfft", "agn_test_irfft", "agn_test_argsort",
              "agn_test_lds_bandwidth"):
        getattr(lib, f).restype = C.c_int


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _check(rc):
    if rc != AGN_OK:
        raise AgnError(rc, lib().agn_last_error().decode())


_F64 = ("torch.float64",)
_F32 = ("torch.float32",)
_I32 = ("torch.int32", "torch.uint32")
_I64 = ("torch.int64", "torch.uint64")


def _buf(t, name="tensor", dtypes=None, need=0, device=None):
    """Device pointer of t, after checking that it is a contiguous GPU tensor
    (on `device` if given) of one of `dtypes` with at least `need` elements.
    The C ABI takes plain pointers and cannot see a buffer's extent, so the
    extents it will touch are checked here; None passes through as NULL."""
    if t is None:
        return None
    if not t.is_cuda:
        raise AgnError(AGN_EINVAL, f"{name}: expected a GPU tensor")
    if not t.is_contiguous():
        raise AgnError(AGN_EINVAL, f"{name}: expected a contiguous tensor")
    if device is not None and t.device.index != device:
        raise AgnError(AGN_EINVAL, f"{name}: tensor on cuda:{t.device.index}, context on cuda:{device}")
    if dtypes is not None and str(t.dtype) not in dtypes:
        raise AgnError(AGN_EINVAL, f"{name}: dtype {t.dtype}, expected {' or '.join(dtypes)}")
    if t.numel() < need:
        raise AgnError(AGN_EINVAL, f"{name}: {t.numel()} elements, at least {need} needed")
    return C.c_void_p(t.data_ptr())


def _wp(prec):
    """Tensor dtype of the working precision (None for an unknown one: the
    library rejects it)."""
    return _F32 if prec == AGN_FP32 else _F64 if prec == AGN_FP64 else None


def _extent(n, offset, per=None):
    """Elements a batch touches: max over curves of offset + per(n) (curves
    with a negative length or offset are left to the library to reject)."""
    n = np.asarray(n, dtype=np.int64)
    o = np.asarray(offset, dtype=np.int64)
    if n.size == 0:
        return 0
    k = n if per is None else per(n)
    return int(np.max(np.where((o >= 0) & (n >= 0), o + k, 0)))


@functools.lru_cache(maxsize=256)
def _nbins_one(n, dex):
    if not (dex > 0.0) or not agn_supported_n(n) or n < 4:
        return 0  # the library rejects the call
    return agn_log_bin_count(n, dex)


def _nbins(n, dex):
    """Log-bin counts of an array of lengths."""
    u, inv = np.unique(np.asarray(n, dtype=np.int64), return_inverse=True)
    return np.array([_nbins_one(int(k), float(dex)) for k in u], dtype=np.int64)[inv.reshape(-1)]


def _stream(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


class Context:
    """agn_ctx on one device (twiddle tables per length and precision)."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = C.c_void_p()
        _check(lib().agn_ctx_create(self.device, C.byref(h)))
        self.handle = h

    def set_profiling(self, on: bool):
        _check(lib().agn_ctx_set_profiling(self.handle, 1 if on else 0))

    def set_lookback_polls(self, polls: int):
        """Look-back wait limit of the multi-pass sort (0: default; < 0: every
        wait gives up at once, for failure-handling tests)."""
        _check(lib().agn_ctx_set_lookback_polls(self.handle, int(polls)))

    def kernel_times(self, reset: bool = True):
        """{kernel name: (total ms, launches)} of the launches timed so far."""
        out = {}
        for name in lib().agn_ctx_kernel_names().decode().split(","):
            ms, cnt = C.c_double(), C.c_int64()
            _check(lib().agn_ctx_kernel_time(self.handle, name.encode(), C.byref(ms), C.byref(cnt), 0))
            out[name] = (ms.value, cnt.value)
        if reset:
            ms, cnt = C.c_double(), C.c_int64()
            _check(lib().agn_ctx_kernel_time(self.handle, b"", C.byref(ms), C.byref(cnt), 1))
        return out

    def close(self):
        if self.handle:
            lib().agn_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def agn_supported_n(n: int) -> bool:
    return bool(lib().agn_supported_n(int(n)))


def agn_spectrum_workspace_size(n: int) -> int:
    b = C.c_size_t()
    _check(lib().agn_spectrum_workspace_size(int(n), C.byref(b)))
    return b.value


def agn_workspace_size(n: int, prec: int) -> int:
    b = C.c_size_t()
    _check(lib().agn_workspace_size(int(n), int(prec), C.byref(b)))
    return b.value


def agn_batch_workspace_size(n, prec: int) -> int:
    n = np.ascontiguousarray(n, dtype=np.int64)
    b = C.c_size_t()
    _check(lib().agn_batch_workspace_size(len(n), n.ctypes.data_as(C.c_void_p), int(prec),
                                          C.byref(b)))
    return b.value


def agn_psd_spectrum(ctx: Context, params, n, dt, seed, curve_id, prec, amp_out, ws, stream=None):
    dv = ctx.device
    _check(lib().agn_psd_spectrum(ctx.handle, C.byref(params), int(n), float(dt), int(seed),
                                  int(curve_id), int(prec), _buf(amp_out, "amp_out", _wp(prec), int(n) // 2 + 1, dv),
                                  _buf(ws, "ws", None, 0, dv),
                                  ws.numel() * ws.element_size(), _stream(stream, ctx.device)))


def agn_psd_spectrum_noalloc(ctx: Context, params, n, dt, seed, curve_id, prec, amp_out, stream=None):
    """agn_psd_spectrum on the library's own device array (no workspace, no allocation)."""
    dv = ctx.device
    _check(lib().agn_psd_spectrum_noalloc(ctx.handle, C.byref(params), int(n), float(dt), int(seed),
                                          int(curve_id), int(prec),
                                          _buf(amp_out, "amp_out", _wp(prec), int(n) // 2 + 1, dv),
                                          _stream(stream, ctx.device)))


def agn_lc_iterate(ctx: Context, amp, x0, n, iters, tol, prec, x_out, delta_out=None,
                   iters_done=None, rank_out=None, ws=None, stream=None):
    dv, k = ctx.device, max(int(n), 0)
    _check(lib().agn_lc_iterate(ctx.handle, _buf(amp, "amp", _wp(prec), k // 2 + 1, dv),
                                _buf(x0, "x0", _F64, k, dv), int(n), int(iters), float(tol),
                                int(prec), _buf(x_out, "x_out", _F64, k, dv),
                                _buf(delta_out, "delta_out", _F64, max(int(iters), 0), dv),
                                _buf(iters_done, "iters_done", _I32, 1, dv),
                                _buf(rank_out, "rank_out", _I32, k, dv), _buf(ws, "ws", None, 0, dv),
                                0 if ws is None else ws.numel() * ws.element_size(),
                                _stream(stream, ctx.device)))


def agn_lc_generate(ctx: Context, params, erdf, n, dt, iters, tol, seed, curve_id, prec, x_out,
                    delta_out=None, iters_done=None, ws=None, stream=None):
    dv, k = ctx.device, max(int(n), 0)
    _check(lib().agn_lc_generate(ctx.handle, C.byref(params), _buf(erdf, "erdf", _F64, k, dv), int(n), float(dt),
                                 int(iters), float(tol), int(seed), int(curve_id), int(prec),
                                 _buf(x_out, "x_out", _F64, k, dv),
                                 _buf(delta_out, "delta_out", _F64, max(int(iters), 0), dv),
                                 _buf(iters_done, "iters_done", _I32, 1, dv), _buf(ws, "ws", None, 0, dv),
                                 0 if ws is None else ws.numel() * ws.element_size(),
                                 _stream(stream, ctx.device)))


def agn_lc_generate_batch(ctx: Context, n, offset, params, dt, iters, seed, curve_id, erdf, tol,
                          prec, x_out, delta_out=None, iters_done=None, ws=None, stream=None):
    """n, offset, dt, iters, seed, curve_id: host sequences; params: sequence of
    agn_psd_params; erdf, x_out, delta_out, iters_done, ws: GPU tensors."""
    nc = len(n)
    n = np.ascontiguousarray(n, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    seed = np.ascontiguousarray(seed, dtype=np.uint64)
    curve_id = np.ascontiguousarray(curve_id, dtype=np.uint32)
    parr = (agn_psd_params * nc)(*params)
    vp = C.c_void_p
    _check(lib().agn_lc_generate_batch(
        ctx.handle, nc, n.ctypes.data_as(vp), offset.ctypes.data_as(vp), C.cast(parr, vp),
        dt.ctypes.data_as(vp), iters.ctypes.data_as(vp), seed.ctypes.data_as(vp),
        curve_id.ctypes.data_as(vp), *_batch_bufs(ctx, n, offset, iters, erdf, x_out, delta_out, iters_done, tol,
                                                  prec),
        _buf(ws, "ws", None, 0, ctx.device), 0 if ws is None else ws.numel() * ws.element_size(),
        _stream(stream, ctx.device)))


def _batch_bufs(ctx, n, offset, iters, erdf, x_out, delta_out, iters_done, tol, prec, *extra):
    """The device-buffer arguments shared by the batch entry points, checked
    against the extents the batch touches."""
    dv = ctx.device
    ext = _extent(n, offset)
    rows = len(n) * (int(np.max(iters)) if len(iters) else 0)
    return (_buf(erdf, "erdf", _F64, ext, dv), float(tol), int(prec), _buf(x_out, "x_out", _F64, ext, dv),
            _buf(delta_out, "delta_out", _F64, max(rows, 0), dv), _buf(iters_done, "iters_done", _I32, len(n), dv),
            *[int(e) for e in extra])


AGN_PLAN_GRAPH = 1
AGN_PLAN_AUTOTUNE = 2
AGN_PLAN_LARGE_SORT_TILE = 4
AGN_PLAN_NARROW_FFT = 8


class BatchPlan:
    """Owns an agn_batch_plan and keeps the tensors it points to alive."""

    def __init__(self, ctx, handle, keep):
        self.ctx = ctx
        self.handle = handle
        self._keep = keep

    def info(self):
        b, g, u = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().agn_batch_plan_info(self.handle, C.byref(b), C.byref(g), C.byref(u)))
        t, f = C.c_int32(), C.c_int32()
        _check(lib().agn_batch_plan_tuning(self.handle, None, C.byref(t), C.byref(f)))
        return {"branches": b.value, "groups": g.value, "graph": bool(u.value), "sort_tile": t.value,
                "fft_cols": f.value}

    def close(self):
        if self.handle:
            _check(lib().agn_batch_plan_destroy(self.handle))
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def agn_batch_plan_create(ctx: Context, n, offset, params, dt, iters, seed, curve_id, erdf, tol, prec,
                          x_out, delta_out=None, iters_done=None, flags=0, branches=0, ws=None, stream=None):
    """Arguments of agn_lc_generate_batch plus flags (AGN_PLAN_GRAPH,
    AGN_PLAN_AUTOTUNE) and branches; returns a BatchPlan."""
    nc = len(n)
    n = np.ascontiguousarray(n, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    seed = np.ascontiguousarray(seed, dtype=np.uint64)
    curve_id = np.ascontiguousarray(curve_id, dtype=np.uint32)
    parr = (agn_psd_params * nc)(*params)
    vp = C.c_void_p
    out = vp()
    _check(lib().agn_batch_plan_create(
        ctx.handle, nc, n.ctypes.data_as(vp), offset.ctypes.data_as(vp), C.cast(parr, vp),
        dt.ctypes.data_as(vp), iters.ctypes.data_as(vp), seed.ctypes.data_as(vp),
        curve_id.ctypes.data_as(vp), *_batch_bufs(ctx, n, offset, iters, erdf, x_out, delta_out, iters_done, tol,
                                                  prec, flags, branches),
        _buf(ws, "ws", None, 0, ctx.device), 0 if ws is None else ws.numel() * ws.element_size(),
        _stream(stream, ctx.device), C.byref(out)))
    return BatchPlan(ctx, out, (erdf, x_out, delta_out, iters_done, ws))


def agn_batch_plan_launch(plan: BatchPlan, stream=None):
    if not plan.handle:
        raise AgnError(int(-1), "plan is closed")
    _check(lib().agn_batch_plan_launch(plan.handle, _stream(stream, plan.ctx.device)))


def agn_log_bin_count(n, dex) -> int:
    c = C.c_int32()
    _check(lib().agn_log_bin_count(int(n), float(dex), C.byref(c)))
    return c.value


def agn_periodogram_workspace_size(n, dex=0.0) -> int:
    n = np.ascontiguousarray(n, dtype=np.int64)
    b = C.c_size_t()
    _check(lib().agn_periodogram_workspace_size(len(n), n.ctypes.data_as(C.c_void_p), float(dex), C.byref(b)))
    return b.value


def agn_periodogram_batch(ctx: Context, n, offset, x, p_offset, P_out, dex=0.0, b_offset=None, bins_out=None,
                          ws=None, stream=None):
    """n, offset, p_offset, b_offset: host sequences; x, P_out, bins_out, ws: GPU tensors."""
    vp = C.c_void_p
    nc = len(n)
    n = np.ascontiguousarray(n, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    p_offset = np.ascontiguousarray(p_offset, dtype=np.int64)
    bo = None if b_offset is None else np.ascontiguousarray(b_offset, dtype=np.int64)
    dv = ctx.device
    _check(lib().agn_periodogram_batch(
        ctx.handle, nc, n.ctypes.data_as(vp), offset.ctypes.data_as(vp), _buf(x, "x", _F64, _extent(n, offset), dv),
        p_offset.ctypes.data_as(vp), _buf(P_out, "P_out", _F64, _extent(n, p_offset, lambda k: k // 2 + 1), dv),
        float(dex), None if bo is None else bo.ctypes.data_as(vp),
        _buf(bins_out, "bins_out", _F64, 0 if bo is None else _extent(n, bo, lambda k: _nbins(k, float(dex))), dv),
        _buf(ws, "ws", None, 0, dv),
        0 if ws is None else ws.numel() * ws.element_size(), _stream(stream, ctx.device)))


AGN_SF_LINEAR, AGN_SF_MAGNITUDE = 0, 1


def agn_psd_fit_workspace_size(n, dex) -> int:
    n = np.ascontiguousarray(n, dtype=np.int64)
    b = C.c_size_t()
    _check(lib().agn_psd_fit_workspace_size(len(n), n.ctypes.data_as(C.c_void_p), float(dex), C.byref(b)))
    return b.value


def agn_psd_fit_batch(ctx: Context, n, dt, params, dex, b_offset, bins, fit_out, ws=None, stream=None):
    """n, dt, params, b_offset: host sequences; bins, fit_out (n_curves x 4 float64), ws: GPU tensors."""
    vp = C.c_void_p
    nc = len(n)
    n = np.ascontiguousarray(n, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    bo = np.ascontiguousarray(b_offset, dtype=np.int64)
    parr = (agn_psd_params * max(nc, 1))(*params)
    dv = ctx.device
    _check(lib().agn_psd_fit_batch(ctx.handle, nc, n.ctypes.data_as(vp), dt.ctypes.data_as(vp), parr, float(dex),
                                   bo.ctypes.data_as(vp),
                                   _buf(bins, "bins", _F64, _extent(n, bo, lambda k: _nbins(k, float(dex))), dv),
                                   _buf(fit_out, "fit_out", _F64, 4 * nc, dv), _buf(ws, "ws", None, 0, dv),
                                   0 if ws is None else ws.numel() * ws.element_size(), _stream(stream, ctx.device)))


def agn_lag_stats_workspace_size(n, lags, n_thr=0, units=AGN_SF_LINEAR):
    vp = C.c_void_p
    n = np.ascontiguousarray(n, dtype=np.int64)
    lags = np.ascontiguousarray(lags, dtype=np.int64)
    out = C.c_size_t(0)
    _check(lib().agn_lag_stats_workspace_size(len(n), n.ctypes.data_as(vp), len(lags), lags.ctypes.data_as(vp),
                                              int(n_thr), int(units), C.byref(out)))
    return out.value


def agn_lag_stats_batch(ctx: Context, n, offset, x, lags, units=AGN_SF_LINEAR, sf2_out=None, rep_out=None,
                        dm_ref=(), lam_cut=0.0, exceed_out=None, pairs_out=None, ws=None, stream=None):
    """n, offset, lags, dm_ref: host sequences; x, outputs, ws: GPU tensors (outputs float64 / uint64 or int64)."""
    vp = C.c_void_p
    n = np.ascontiguousarray(n, dtype=np.int64)
    offset = np.ascontiguousarray(offset, dtype=np.int64)
    lags = np.ascontiguousarray(lags, dtype=np.int64)
    dm = np.ascontiguousarray(dm_ref, dtype=np.float64)
    dv, items = ctx.device, len(n) * len(lags)
    _check(lib().agn_lag_stats_batch(
        ctx.handle, len(n), n.ctypes.data_as(vp), offset.ctypes.data_as(vp), _buf(x, "x", _F64, _extent(n, offset), dv),
        len(lags), lags.ctypes.data_as(vp), int(units), _buf(sf2_out, "sf2_out", _F64, items, dv),
        _buf(rep_out, "rep_out", _F64, len(lags), dv), len(dm), dm.ctypes.data_as(vp) if len(dm) else None,
        float(lam_cut), _buf(exceed_out, "exceed_out", _I64, items * len(dm), dv),
        _buf(pairs_out, "pairs_out", _I64, items, dv), _buf(ws, "ws", None, 0, dv),
        0 if ws is None else ws.numel() * ws.element_size(), _stream(stream, ctx.device)))


def agn_erdf_draw(ctx: Context, params, n, seed, curve_id, out, stream=None):
    _check(lib().agn_erdf_draw(ctx.handle, C.byref(params), int(n), int(seed), int(curve_id),
                               _buf(out, "out", _F64, max(int(n), 0), ctx.device),
                               _stream(stream, ctx.device)))


def agn_pdf_draw(ctx: Context, params, n, seed, curve_id, out, stream=None):
    _check(lib().agn_pdf_draw(ctx.handle, C.byref(params), int(n), int(seed), int(curve_id),
                              _buf(out, "out", _F64, max(int(n), 0), ctx.device),
                              _stream(stream, ctx.device)))


def agn_pdf_slice(ctx: Context, params, n, n_chains, burn, seed, curve_id, out, stream=None):
    _check(lib().agn_pdf_slice(ctx.handle, C.byref(params), int(n), int(n_chains), int(burn), int(seed),
                               int(curve_id), _buf(out, "out", _F64, max(int(n), 0), ctx.device),
                               _stream(stream, ctx.device)))


def agn_test_philox(key0, key1, ctr0, n_blocks, out, stream=None, device=0):
    _check(lib().agn_test_philox(int(key0) & (2**64 - 1), int(key1) & (2**64 - 1),
                                 int(ctr0) & (2**64 - 1), int(n_blocks),
                                 _buf(out, "out", _I64, 4 * max(int(n_blocks), 0), device),
                                 _stream(stream, device)))


AGN_TEST_PATH_LDS, AGN_TEST_PATH_HBM = 0, 1


def agn_test_workspace_size(n: int, prec: int, path: int) -> int:
    b = C.c_size_t()
    _check(lib().agn_test_workspace_size(int(n), int(prec), int(path), C.byref(b)))
    return b.value


def agn_test_rfft(ctx: Context, x, n, prec, path, X_out, ws, stream=None):
    """X_out: float64 tensor of 2 (n/2 + 1) values, (re, im) interleaved."""
    dv, k = ctx.device, max(int(n), 0)
    _check(lib().agn_test_rfft(ctx.handle, _buf(x, "x", _F64, k, dv), int(n), int(prec), int(path),
                               _buf(X_out, "X_out", _F64, 2 * (k // 2 + 1), dv), _buf(ws, "ws", None, 0, dv),
                               0 if ws is None else ws.numel() * ws.element_size(), _stream(stream, dv)))


def agn_test_irfft(ctx: Context, Y, n, prec, path, y_out, ws, stream=None):
    """Y: float64 tensor of 2 (n/2 + 1) values, (re, im) interleaved."""
    dv, k = ctx.device, max(int(n), 0)
    _check(lib().agn_test_irfft(ctx.handle, _buf(Y, "Y", _F64, 2 * (k // 2 + 1), dv), int(n), int(prec),
                                int(path), _buf(y_out, "y_out", _F64, k, dv), _buf(ws, "ws", None, 0, dv),
                                0 if ws is None else ws.numel() * ws.element_size(), _stream(stream, dv)))


def agn_test_argsort(ctx: Context, y, n, prec, path, rank_out, ws, stream=None):
    dv, k = ctx.device, max(int(n), 0)
    _check(lib().agn_test_argsort(ctx.handle, _buf(y, "y", _F64, k, dv), int(n), int(prec), int(path),
                                  _buf(rank_out, "rank_out", _I32, k, dv), _buf(ws, "ws", None, 0, dv),
                                  0 if ws is None else ws.numel() * ws.element_size(), _stream(stream, dv)))


def agn_test_lds_bandwidth(blocks: int, reps: int, out, stream=None, device=0) -> float:
    """Measured LDS read bandwidth in bytes/s (blocks x reps x 64 KB read)."""
    sec = C.c_double()
    _check(lib().agn_test_lds_bandwidth(int(blocks), int(reps), _buf(out, "out", _F32, int(blocks) * 1024, device),
                                        C.byref(sec), _stream(stream, device)))
    return int(blocks) * int(reps) * 65536 / sec.value
