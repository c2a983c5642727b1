"""ctypes binding of the C ABI in include/fstat.h.

Argument marshalling only: torch supplies device memory and streams, every
step of the computation runs in the HIP library.  If the library is missing
the functions raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfstat.so")
MAX_DET = 4
TEMPLATE_STRIDE = 8
TEMPLATE_STRIDE_KEPLER = 10
PLAN_KEPLER = 1

FSTAT_OK, FSTAT_EINVAL, FSTAT_EUNSUPPORTED, FSTAT_EWORKSPACE, FSTAT_EHIP, FSTAT_EINTERNAL = \
    0, -1, -2, -3, -4, -5

EXPORTED = ("fstat_plan_create", "fstat_plan_destroy", "fstat_workspace_size",
            "fstat_antenna_moments", "fstat_compute_2f", "fstat_compute_2f_batched",
            "fstat_compute_2f_profiled", "fstat_resample", "fstat_sync_check",
            "fstat_last_error", "fstat_version", "fstat_search_create", "fstat_search_destroy",
            "fstat_search_info", "fstat_search_run", "fstat_search_run_profiled",
            "fstat_grad_workspace_size", "fstat_compute_2f_grad", "fstat_plan_info",
            "fstat_grad_bin_workspace_size", "fstat_compute_2f_grad_bin", "fstat_autotune",
            "fstat_search_run_candidates", "fstat_batch_create", "fstat_batch_destroy",
            "fstat_batch_run", "fstat_flagged_count", "fstat_sfts_to_series",
            "fstat_compute_2f_grad_bin_noalloc", "fstat_sinc_halfwidth_for",
            "fstat_autotune_search")
GRAD_PARAMS = ("df", "f1dot", "alpha", "delta", "asini", "porb", "tp")
# template-row column of each gradient parameter
GRAD_COLUMNS = (2, 3, 0, 1, 5, 6, 7)
SEARCH_GRAPH = 1
SEARCH_ACCUMULATE = 2


class FstatDetector(ctypes.Structure):
    _fields_ = [("lat", ctypes.c_double), ("lon", ctypes.c_double), ("az_x", ctypes.c_double),
                ("az_y", ctypes.c_double), ("t0", ctypes.c_double), ("n", ctypes.c_int64),
                ("noise_var", ctypes.c_double)]


class FstatPlanDesc(ctypes.Structure):
    _fields_ = [("ndet", ctypes.c_int32), ("sinc_halfwidth", ctypes.c_int32),
                ("det", FstatDetector * MAX_DET), ("dt", ctypes.c_double),
                ("f_het", ctypes.c_double), ("t_ref", ctypes.c_double), ("tau0", ctypes.c_double),
                ("max_delay", ctypes.c_double), ("sid_angle0", ctypes.c_double),
                ("sid_rate", ctypes.c_double), ("n_fft", ctypes.c_int64),
                ("bin_lo", ctypes.c_int64), ("n_bins", ctypes.c_int64),
                ("tune_col_log_len", ctypes.c_int32), ("tune_col_lines", ctypes.c_int32),
                ("tune_row_lines", ctypes.c_int32), ("tune_fft_radix", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class FstatInputs(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p * MAX_DET), ("valid", ctypes.c_void_p * MAX_DET),
                ("ephem", ctypes.c_void_p * MAX_DET), ("n_eph", ctypes.c_int64),
                ("eph_t0", ctypes.c_double), ("eph_dt", ctypes.c_double),
                ("moments", ctypes.c_void_p)]


class FstatSftDesc(ctypes.Structure):
    _fields_ = [("t_start", ctypes.c_double), ("t_sft", ctypes.c_double),
                ("n_sft", ctypes.c_int64), ("k0", ctypes.c_int64), ("n_bins", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class FstatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fstat status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfstat.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FstatError(FSTAT_EUNSUPPORTED,
                         f"{path} not built; run __graft_entry__.build() or "
                         "python paper_2201_00451_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.fstat_plan_create.argtypes = [ctypes.POINTER(FstatPlanDesc), ctypes.POINTER(vp)]
    lib.fstat_plan_destroy.argtypes = [vp]
    lib.fstat_plan_destroy.restype = None
    lib.fstat_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    lib.fstat_antenna_moments.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, vp, sz, vp]
    for name in ("fstat_compute_2f", "fstat_compute_2f_batched"):
        getattr(lib, name).argtypes = [vp, ctypes.POINTER(FstatInputs), vp, i64, vp, vp, vp, sz, vp]
    lib.fstat_compute_2f_profiled.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, i64, vp, vp,
                                              sz, i64, vp, ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(ctypes.c_int64)]
    lib.fstat_resample.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, i64, vp, vp, sz, vp]
    lib.fstat_search_create.argtypes = [vp, vp, i64, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(vp)]
    lib.fstat_search_destroy.argtypes = [vp]
    lib.fstat_search_destroy.restype = None
    lib.fstat_search_info.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]
    lib.fstat_search_run.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, vp, vp, vp, sz, vp]
    lib.fstat_search_run_candidates.argtypes = [vp, ctypes.POINTER(FstatInputs), vp,
                                                ctypes.c_float, vp, i64, vp, vp, vp, sz, vp]
    lib.fstat_search_run_profiled.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, vp, vp, sz, vp,
                                              ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(ctypes.c_int64)]
    lib.fstat_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.fstat_autotune.argtypes = [ctypes.POINTER(FstatPlanDesc), ctypes.POINTER(FstatInputs),
                                   vp, i64, vp, vp, sz, vp, ctypes.POINTER(FstatPlanDesc),
                                   ctypes.POINTER(ctypes.c_float)]
    lib.fstat_autotune_search.argtypes = [ctypes.POINTER(FstatPlanDesc),
                                          ctypes.POINTER(FstatInputs), vp, vp, i64,
                                          ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_char_p,
                                          vp, ctypes.POINTER(FstatPlanDesc),
                                          ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.fstat_grad_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    lib.fstat_grad_bin_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    lib.fstat_compute_2f_grad_bin.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, i64, vp, vp,
                                              vp, vp, sz, vp]
    lib.fstat_compute_2f_grad.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, i64, vp, vp, vp,
                                          vp, sz, vp]
    lib.fstat_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(vp)]
    lib.fstat_batch_destroy.argtypes = [vp]
    lib.fstat_batch_destroy.restype = None
    lib.fstat_batch_run.argtypes = [vp, ctypes.POINTER(ctypes.POINTER(FstatInputs)),
                                    ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(sz), vp]
    lib.fstat_flagged_count.argtypes = [vp, sz, vp, ctypes.POINTER(i64)]
    lib.fstat_sinc_halfwidth_for.argtypes = [ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_double)]
    lib.fstat_compute_2f_grad_bin_noalloc.argtypes = [vp, ctypes.POINTER(FstatInputs), vp, i64,
                                                      vp, vp, vp, vp]
    lib.fstat_sfts_to_series.argtypes = [ctypes.POINTER(FstatSftDesc), vp, vp, vp, vp, vp]
    lib.fstat_sync_check.argtypes = [vp]
    lib.fstat_last_error.restype = ctypes.c_char_p
    lib.fstat_last_error.argtypes = []
    lib.fstat_version.restype = ctypes.c_char_p
    lib.fstat_version.argtypes = []
    for name in EXPORTED:
        if name not in ("fstat_plan_destroy", "fstat_last_error", "fstat_version",
                        "fstat_search_destroy", "fstat_batch_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status != FSTAT_OK:
        raise FstatError(status, load_library().fstat_last_error().decode())


def last_error() -> str:
    return load_library().fstat_last_error().decode()


def version() -> str:
    return load_library().fstat_version().decode()


def make_plan_desc(ds, tune=None) -> FstatPlanDesc:
    """Plan descriptor from a search description (see synth.Dataset).
    tune: optional dict of tune_col_log_len / tune_col_lines / tune_row_lines."""
    d = FstatPlanDesc()
    d.ndet = len(ds.detectors)
    d.sinc_halfwidth = int(ds.sinc_halfwidth)
    for i, det in enumerate(ds.detectors):
        d.det[i] = FstatDetector(det.lat, det.lon, det.az_x, det.az_y, det.t0, det.n, det.noise_var)
    d.dt, d.f_het, d.t_ref, d.tau0 = ds.dt, ds.f_het, ds.t_ref, ds.tau0
    d.max_delay = ds.max_delay
    d.sid_angle0 = ds.ephem_model["sidereal_angle0_rad"]
    d.sid_rate = ds.ephem_model["sidereal_rate_rad_s"]
    d.n_fft, d.bin_lo, d.n_bins = ds.n_fft, ds.bin_lo, ds.n_bins
    # rows of ten: Keplerian orbits (eccentricity, argument of periapsis)
    kepler = np.asarray(ds.templates).shape[1] == TEMPLATE_STRIDE_KEPLER
    d.flags = PLAN_KEPLER if kepler else 0
    for k, v in (tune or {}).items():
        setattr(d, k, int(v))
    return d


class Plan:
    """Owns an fstat_plan handle."""

    def __init__(self, desc: FstatPlanDesc):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.fstat_plan_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.desc = desc

    def workspace_size(self, batch: int = 1) -> int:
        out = ctypes.c_size_t()
        _check(load_library().fstat_workspace_size(self.handle, int(batch), ctypes.byref(out)))
        return int(out.value)

    def info(self):
        """(k_pad, log2 column length, log2 row length) of the plan."""
        k, lc, lr = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().fstat_plan_info(self.handle, ctypes.byref(k), ctypes.byref(lc),
                                              ctypes.byref(lr)))
        return int(k.value), int(lc.value), int(lr.value)

    def grad_bin_workspace_size(self, batch: int = 1) -> int:
        out = ctypes.c_size_t()
        _check(load_library().fstat_grad_bin_workspace_size(self.handle, int(batch),
                                                            ctypes.byref(out)))
        return int(out.value)

    def grad_workspace_size(self, batch: int = 1) -> int:
        out = ctypes.c_size_t()
        _check(load_library().fstat_grad_workspace_size(self.handle, int(batch),
                                                        ctypes.byref(out)))
        return int(out.value)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fstat_plan_destroy(self.handle)
            self.handle = None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class DeviceData:
    """Device copies of a data set (copied once), the antenna moments and a
    workspace, bound to a plan.  ``ds`` follows synth.Dataset's fields."""

    def __init__(self, ds, device="cuda:0", batch=1, stream=None, tune=None):
        import torch
        if not torch.cuda.is_available():
            raise FstatError(FSTAT_EUNSUPPORTED, "no HIP device visible to torch")
        self.device = torch.device(device)
        self.plan = Plan(make_plan_desc(ds, tune))
        self.stride = (TEMPLATE_STRIDE_KEPLER if self.plan.desc.flags & PLAN_KEPLER
                       else TEMPLATE_STRIDE)
        self.ndet = len(ds.detectors)
        self.n_fft, self.n_bins = int(ds.n_fft), int(ds.n_bins)
        dev = self.device
        self.x = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to(dev)
                  for x in ds.x]
        self.valid = [torch.from_numpy(np.ascontiguousarray(v, dtype=np.uint8)).to(dev)
                      for v in ds.valid]
        self.ephem = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(dev)
                      for t in ds.eph_tables]
        self.moments = torch.zeros((self.ndet, 10), dtype=torch.float64, device=dev)
        self.inputs = FstatInputs()
        for i in range(self.ndet):
            self.inputs.x[i] = self.x[i].data_ptr()
            self.inputs.valid[i] = self.valid[i].data_ptr()
            self.inputs.ephem[i] = self.ephem[i].data_ptr()
        self.inputs.n_eph = int(ds.eph_tables[0].shape[0])
        self.inputs.eph_t0, self.inputs.eph_dt = float(ds.eph_t0), float(ds.eph_dt)
        self.inputs.moments = self.moments.data_ptr()
        self.set_batch(batch)
        antenna_moments(self, stream)

    def set_batch(self, batch):
        import torch
        nbytes = self.plan.workspace_size(batch)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.batch = batch


def antenna_moments(dd: DeviceData, stream=None):
    _check(load_library().fstat_antenna_moments(
        dd.plan.handle, ctypes.byref(dd.inputs), _ptr(dd.moments), _ptr(dd.ws), dd.ws.numel(),
        _stream_ptr(stream)))
    return dd.moments


def _templates(dd, templates):
    import torch
    t = torch.as_tensor(templates, dtype=torch.float64)
    if t.dim() != 2 or t.shape[1] != dd.stride:
        raise FstatError(FSTAT_EINVAL, f"templates must have shape [n, {dd.stride}]")
    return t.to(dd.device).contiguous()


def compute_2f(dd: DeviceData, templates, fafb=False, batched=False, out=None, stream=None):
    """2F [n, n_bins] float32 on the device (and Fa, Fb [n, 2, n_bins] complex64)."""
    import torch
    tm = _templates(dd, templates)
    n = tm.shape[0]
    tf = out if out is not None else torch.empty((n, dd.n_bins), dtype=torch.float32,
                                                 device=dd.device)
    fab = torch.empty((n, 2, dd.n_bins), dtype=torch.complex64, device=dd.device) if fafb else None
    fn = load_library().fstat_compute_2f_batched if batched else load_library().fstat_compute_2f
    _check(fn(dd.plan.handle, ctypes.byref(dd.inputs), _ptr(tm), n, _ptr(tf), _ptr(fab),
              _ptr(dd.ws), dd.ws.numel(), _stream_ptr(stream)))
    return (tf, fab) if fafb else tf


def compute_2f_batched(dd: DeviceData, templates, fafb=False, out=None, stream=None):
    return compute_2f(dd, templates, fafb=fafb, batched=True, out=out, stream=stream)


KERNELS = ("prologue", "resample", "fft_columns", "fft_rows_2f")


def compute_2f_profiled(dd: DeviceData, templates, max_batch=None, out=None, stream=None):
    """compute_2f_batched plus per-kernel device time (ms) and launch counts.
    Synchronises the stream."""
    import torch
    tm = _templates(dd, templates)
    n = tm.shape[0]
    tf = out if out is not None else torch.empty((n, dd.n_bins), dtype=torch.float32,
                                                 device=dd.device)
    ms = (ctypes.c_float * 4)()
    cnt = (ctypes.c_int64 * 4)()
    mb = dd.batch if max_batch is None else int(max_batch)
    _check(load_library().fstat_compute_2f_profiled(
        dd.plan.handle, ctypes.byref(dd.inputs), _ptr(tm), n, _ptr(tf), _ptr(dd.ws), dd.ws.numel(),
        mb, _stream_ptr(stream), ms, cnt))
    return tf, {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNELS)}


def resample(dd: DeviceData, templates, stream=None):
    """Weighted resampled series y [n, 2, n_fft] complex64 (diagnostic)."""
    import torch
    tm = _templates(dd, templates)
    n = tm.shape[0]
    y = torch.empty((n, 2, dd.n_fft), dtype=torch.complex64, device=dd.device)
    _check(load_library().fstat_resample(dd.plan.handle, ctypes.byref(dd.inputs), _ptr(tm), n,
                                         _ptr(y), _ptr(dd.ws), dd.ws.numel(), _stream_ptr(stream)))
    return y


def compute_2f_grad(dd: DeviceData, templates, grad_twoF, want_twoF=False, batch=4,
                    stream=None):
    """d(sum grad_twoF * 2F)/d theta per template, theta = GRAD_PARAMS:
    float64 [n, 7] on the device (and 2F [n, n_bins] if want_twoF).  The
    adjoint workspace (``batch`` templates in flight) is kept on ``dd``."""
    import torch
    tm = _templates(dd, templates)
    n = tm.shape[0]
    g = torch.as_tensor(grad_twoF, dtype=torch.float32).to(dd.device).contiguous()
    if tuple(g.shape) != (n, dd.n_bins):
        raise FstatError(FSTAT_EINVAL, f"grad_twoF must have shape [{n}, {dd.n_bins}]")
    nbytes = dd.plan.grad_workspace_size(batch)
    if getattr(dd, "grad_ws", None) is None or dd.grad_ws.numel() != nbytes:
        dd.grad_ws = torch.empty(nbytes, dtype=torch.uint8, device=dd.device)
    grad = torch.empty((n, len(GRAD_PARAMS)), dtype=torch.float64, device=dd.device)
    tf = torch.empty((n, dd.n_bins), dtype=torch.float32, device=dd.device) if want_twoF else None
    _check(load_library().fstat_compute_2f_grad(
        dd.plan.handle, ctypes.byref(dd.inputs), _ptr(tm), n, _ptr(g), _ptr(grad), _ptr(tf),
        _ptr(dd.grad_ws), dd.grad_ws.numel(), _stream_ptr(stream)))
    return (grad, tf) if want_twoF else grad


def compute_2f_grad_bin(dd: DeviceData, templates, bins, batch=32, stream=None):
    """Single-bin form: (gradient of 2F at bins[m] for template m, float64
    [n, 7]; 2F at that bin, float32 [n]), both on the device.  No FFT runs."""
    import torch
    tm = _templates(dd, templates)
    n = tm.shape[0]
    b = torch.as_tensor(np.asarray(bins, dtype=np.int64)).to(dd.device).contiguous()
    if tuple(b.shape) != (n,):
        raise FstatError(FSTAT_EINVAL, f"bins must have shape [{n}]")
    nbytes = dd.plan.grad_bin_workspace_size(batch)
    if getattr(dd, "grad_bin_ws", None) is None or dd.grad_bin_ws.numel() != nbytes:
        dd.grad_bin_ws = torch.empty(nbytes, dtype=torch.uint8, device=dd.device)
    grad = torch.empty((n, len(GRAD_PARAMS)), dtype=torch.float64, device=dd.device)
    tf = torch.empty((n,), dtype=torch.float32, device=dd.device)
    _check(load_library().fstat_compute_2f_grad_bin(
        dd.plan.handle, ctypes.byref(dd.inputs), _ptr(tm), n, _ptr(b), _ptr(tf), _ptr(grad),
        _ptr(dd.grad_bin_ws), dd.grad_bin_ws.numel(), _stream_ptr(stream)))
    return grad, tf


def compute_2f_grad_bin_noalloc(dd: DeviceData, templates, bins, stream=None):
    """compute_2f_grad_bin without a workspace argument: the library's static
    device scratch (fstat_compute_2f_grad_bin_noalloc).  Returns (grad [n, 7]
    float64, 2F [n] float32) on the device."""
    import torch
    tm = _templates(dd, templates)
    n = tm.shape[0]
    b = torch.as_tensor(np.asarray(bins, dtype=np.int64)).to(dd.device).contiguous()
    grad = torch.empty((n, len(GRAD_PARAMS)), dtype=torch.float64, device=dd.device)
    tf = torch.empty((n,), dtype=torch.float32, device=dd.device)
    _check(load_library().fstat_compute_2f_grad_bin_noalloc(
        dd.plan.handle, ctypes.byref(dd.inputs), _ptr(tm), n, _ptr(b), _ptr(tf), _ptr(grad),
        _stream_ptr(stream)))
    return grad, tf


def template_rows(params, f2dot=None, kepler=None):
    """Template rows from params [n, 7] in GRAD_PARAMS order (float64): [n, 8],
    or [n, 10] with kepler = (ecc, argp) per row ([n, 2]) for Keplerian plans."""
    import torch
    p = torch.as_tensor(params, dtype=torch.float64)
    width = TEMPLATE_STRIDE if kepler is None else TEMPLATE_STRIDE_KEPLER
    rows = torch.zeros((p.shape[0], width), dtype=torch.float64, device=p.device)
    for i, c in enumerate(GRAD_COLUMNS):
        rows[:, c] = p[:, i]
    if f2dot is not None:
        rows[:, 4] = torch.as_tensor(f2dot, dtype=torch.float64, device=p.device)
    if kepler is not None:
        rows[:, 8:10] = torch.as_tensor(kepler, dtype=torch.float64, device=p.device)
    return rows


def _fstat_fn():
    import torch

    class FStatFn(torch.autograd.Function):
        """2F [n, n_bins] of params [n, 7] (GRAD_PARAMS order; f2dot fixed).
        Forward: fstat_compute_2f_batched.  Backward: fstat_compute_2f_grad
        with the incoming gradient as the bin weights (float64 result)."""

        @staticmethod
        def forward(ctx, params, dd, f2dot):
            rows = template_rows(params.detach(), f2dot)
            ctx.dd, ctx.rows = dd, rows
            return compute_2f_batched(dd, rows)

        @staticmethod
        def backward(ctx, grad_out):
            g = compute_2f_grad(ctx.dd, ctx.rows, grad_out.detach().float())
            return g, None, None

    return FStatFn


_FSTAT_FN = None


def twoF(dd: DeviceData, params, f2dot=None):
    """Differentiable 2F: ``params`` [n, 7] float64 (GRAD_PARAMS order) on the
    device; gradients flow back through the adjoint kernels."""
    global _FSTAT_FN
    if _FSTAT_FN is None:
        _FSTAT_FN = _fstat_fn()
    return _FSTAT_FN.apply(params, dd, f2dot)


def refine(dd: DeviceData, templates, bins, scales, steps=50, lr=0.5, free=None):
    """Gradient-ascent refinement of candidates: maximise 2F in bin bins[m]
    of template m over the free parameters (default: all seven for binary
    rows, df/f1dot/alpha/delta for isolated ones).  The ascent runs on log 2F
    in coordinates scaled by ``scales`` [7] (one metric spacing per
    parameter): u = scales * grad / 2F, capped at unit length, and
    theta += lr * scales * u.  A step is kept only where 2F does not decrease;
    then lr grows by 1.5 (at most 4), else it halves, per candidate.  Every 2F
    and gradient comes from the HIP kernels (the single-bin adjoint: no FFT).
    Returns (rows, 2F at bins) as host arrays."""
    import torch
    rows = torch.as_tensor(np.asarray(templates, dtype=np.float64)).clone()
    n = rows.shape[0]
    bins = torch.as_tensor(np.asarray(bins, dtype=np.int64))
    sc = torch.as_tensor(np.asarray(scales, dtype=np.float64))
    mask = torch.ones((n, 7), dtype=torch.float64)
    mask[rows[:, 5] == 0.0, 4:] = 0.0
    if free is not None:
        keep = torch.tensor([1.0 if p in free else 0.0 for p in GRAD_PARAMS], dtype=torch.float64)
        mask = mask * keep
    step = torch.full((n,), float(lr), dtype=torch.float64)
    cols = list(GRAD_COLUMNS)
    g, tf = compute_2f_grad_bin(dd, rows, bins)
    cur = tf.cpu().double()
    g = g.cpu()
    for _ in range(steps):
        u = sc * g * mask / torch.clamp(cur, min=1.0)[:, None]
        u = u / torch.clamp(torch.linalg.vector_norm(u, dim=1), min=1.0)[:, None]
        trial = rows.clone()
        trial[:, cols] = rows[:, cols] + step[:, None] * sc * u
        g_t, tf_t = compute_2f_grad_bin(dd, trial, bins)
        val = tf_t.cpu().double()
        ok = torch.isfinite(val) & (val >= cur)
        rows[ok] = trial[ok]
        cur = torch.where(ok, val, cur)
        g = torch.where(ok[:, None], g_t.cpu(), g)
        step = torch.where(ok, torch.clamp(step * 1.5, max=4.0), step * 0.5)
    return rows.numpy(), cur.numpy()


TUNE_FIELDS = ("tune_col_log_len", "tune_col_lines", "tune_row_lines", "tune_fft_radix")


def autotune(ds, templates, batch=8, device="cuda:0", stream=None):
    """fstat_autotune on a sample of templates: returns (tune dict, ms) for the
    fastest FFT launch shape of this set-up (pass the dict as ``tune`` to
    DeviceData)."""
    import torch
    dd = DeviceData(ds, device=device, batch=batch)
    tm = _templates(dd, templates)
    n = tm.shape[0]
    tf = torch.empty((n, dd.n_bins), dtype=torch.float32, device=dd.device)
    best = FstatPlanDesc()
    ms = ctypes.c_float()
    _check(load_library().fstat_autotune(ctypes.byref(dd.plan.desc), ctypes.byref(dd.inputs),
                                         _ptr(tm), n, _ptr(tf), _ptr(dd.ws), dd.ws.numel(),
                                         _stream_ptr(stream), ctypes.byref(best),
                                         ctypes.byref(ms)))
    return {k: int(getattr(best, k)) for k in TUNE_FIELDS}, float(ms.value)


def autotune_search(dd: "DeviceData", templates, slots=32, repeats=3, cache=None,
                    stream=None):
    """fstat_autotune_search: the fastest FFT launch shape of this set-up on
    the search path, timed as the median of `repeats` searches of the sample
    `templates` with `slots` slots.  cache: a JSON-lines file (None: the
    library reads FSTAT_AUTOTUNE_CACHE).  Returns (tune dict, median ms,
    from_cache); pass the dict as ``tune`` to DeviceData."""
    import torch
    host = np.ascontiguousarray(np.asarray(templates, dtype=np.float64))
    tm = _templates(dd, host)
    n = tm.shape[0]
    tf = torch.empty((n, dd.n_bins), dtype=torch.float32, device=dd.device)
    best = FstatPlanDesc()
    ms = ctypes.c_float()
    hit = ctypes.c_int32()
    _check(load_library().fstat_autotune_search(
        ctypes.byref(dd.plan.desc), ctypes.byref(dd.inputs),
        host.ctypes.data_as(ctypes.c_void_p), _ptr(tm), n, int(slots), int(repeats), _ptr(tf),
        None if cache is None else str(cache).encode(), _stream_ptr(stream),
        ctypes.byref(best), ctypes.byref(ms), ctypes.byref(hit)))
    return {k: int(getattr(best, k)) for k in TUNE_FIELDS}, float(ms.value), bool(hit.value)


def sfts_to_series(sfts, present, k0, t_sft, t_start=0.0, device="cuda:0", stream=None):
    """Steps (i)-(ii) on the GPU (fstat_sfts_to_series): SFTs [n_sft, K]
    complex64 (host or device) and their presence flags [n_sft] to the
    heterodyned series x [n_sft K] complex64 and its validity [n_sft K] uint8,
    both on the device; also returns (f_het, dt) of the series."""
    import torch
    X = torch.as_tensor(sfts).to(device=device, dtype=torch.complex64).contiguous()
    n_sft, K = X.shape
    pr = None if present is None else torch.as_tensor(
        np.asarray(present, dtype=np.uint8)).to(device).contiguous()
    x = torch.empty(n_sft * K, dtype=torch.complex64, device=device)
    v = torch.empty(n_sft * K, dtype=torch.uint8, device=device)
    d = FstatSftDesc(float(t_start), float(t_sft), int(n_sft), int(k0), int(K), 0)
    _check(load_library().fstat_sfts_to_series(ctypes.byref(d), _ptr(X), _ptr(pr), _ptr(x),
                                                _ptr(v), _stream_ptr(stream)))
    return x, v, (k0 + K / 2) / t_sft, t_sft / K


def sinc_halfwidth_for(band_fraction, tol_2f=1e-3):
    """fstat_sinc_halfwidth_for: (D, worst 2F error) for an accuracy bound."""
    D = ctypes.c_int32()
    err = ctypes.c_double()
    _check(load_library().fstat_sinc_halfwidth_for(float(band_fraction), float(tol_2f),
                                                    ctypes.byref(D), ctypes.byref(err)))
    return int(D.value), float(err.value)


def flagged_count(ws, stream=None) -> int:
    """Templates whose outputs the last call on workspace tensor ``ws`` set
    to NaN (fstat_flagged_count; synchronises the stream)."""
    n = ctypes.c_int64()
    _check(load_library().fstat_flagged_count(_ptr(ws), ws.numel(), _stream_ptr(stream),
                                              ctypes.byref(n)))
    return int(n.value)


def sync_check(stream=None):
    _check(load_library().fstat_sync_check(_stream_ptr(stream)))


def search_workspace_size(dd: DeviceData, templates, slots=8) -> int:
    """Workspace bytes fstat_search_info reports for this bank (host-only:
    plans the bank and destroys the handle)."""
    lib = load_library()
    host = np.ascontiguousarray(np.asarray(templates, dtype=np.float64))
    h = ctypes.c_void_p()
    _check(lib.fstat_search_create(dd.plan.handle, host.ctypes.data_as(ctypes.c_void_p),
                                   host.shape[0], int(slots), 0, ctypes.byref(h)))
    ws = ctypes.c_size_t()
    try:
        _check(lib.fstat_search_info(h, ctypes.byref(ws), None, None))
    finally:
        lib.fstat_search_destroy(h)
    return int(ws.value)


class Search:
    """Grouped path for a template bank (fstat_search_*): templates sharing a
    sky position and orbit are resampled once.  ``templates`` is the bank in
    host memory; the same rows are copied to the device once."""

    def __init__(self, dd: DeviceData, templates, slots=8, graph=False, accumulate=False,
                 workspace=None):
        """workspace: optional device uint8 tensor of at least ws_bytes to use
        instead of a workspace of the search's own (searches run one after
        another on one stream may share one)."""
        import torch
        lib = load_library()
        host = np.ascontiguousarray(np.asarray(templates, dtype=np.float64))
        if host.ndim != 2 or host.shape[1] != dd.stride:
            raise FstatError(FSTAT_EINVAL, f"templates must have shape [n, {dd.stride}]")
        self.dd, self.ntmpl = dd, host.shape[0]
        h = ctypes.c_void_p()
        flags = (SEARCH_GRAPH if graph else 0) | (SEARCH_ACCUMULATE if accumulate else 0)
        _check(lib.fstat_search_create(dd.plan.handle, host.ctypes.data_as(ctypes.c_void_p),
                                       self.ntmpl, int(slots), flags, ctypes.byref(h)))
        self.handle = h
        ws, ng, nc = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.fstat_search_info(h, ctypes.byref(ws), ctypes.byref(ng), ctypes.byref(nc)))
        self.ws_bytes, self.ngroups, self.nchunks = int(ws.value), int(ng.value), int(nc.value)
        self.templates = torch.from_numpy(host).to(dd.device)
        if workspace is not None:
            if workspace.numel() < self.ws_bytes:
                raise FstatError(FSTAT_EWORKSPACE,
                                 f"workspace {workspace.numel()} bytes < {self.ws_bytes}")
            self.ws = workspace
        else:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dd.device)
        self.graph = graph

    def run(self, out=None, fafb=False, stream=None):
        import torch
        dd = self.dd
        tf = out if out is not None else torch.empty((self.ntmpl, dd.n_bins), dtype=torch.float32,
                                                     device=dd.device)
        fab = (torch.empty((self.ntmpl, 2, dd.n_bins), dtype=torch.complex64, device=dd.device)
               if fafb else None)
        _check(load_library().fstat_search_run(self.handle, ctypes.byref(dd.inputs),
                                               _ptr(self.templates), _ptr(tf), _ptr(fab),
                                               _ptr(self.ws), self.ws.numel(), _stream_ptr(stream)))
        return (tf, fab) if fafb else tf

    def run_candidates(self, threshold, capacity=1 << 16, stream=None):
        """Candidate retention (fstat_search_run_candidates): returns a dict with
        the device tensors tmpl, bin (int32), twoF (float32) of the stored
        candidates (unordered), the total count (a Python int: may exceed
        capacity), and per template best_twoF (float32; NaN for a flagged
        template) and best_bin (int64).  Synchronises the stream."""
        import torch
        dd = self.dd
        cand = torch.empty((max(int(capacity), 1), 4), dtype=torch.int32, device=dd.device)
        count = torch.empty(1, dtype=torch.int64, device=dd.device)
        best = torch.empty(max(self.ntmpl, 1), dtype=torch.int64, device=dd.device)
        _check(load_library().fstat_search_run_candidates(
            self.handle, ctypes.byref(dd.inputs), _ptr(self.templates), float(threshold),
            _ptr(cand), int(capacity), _ptr(count), _ptr(best), _ptr(self.ws), self.ws.numel(),
            _stream_ptr(stream)))
        n = int(count.item())
        kept = cand[:min(n, int(capacity))]
        flagged = best == -1
        hi = (best >> 32) & 0xFFFFFFFF
        best_twoF = hi.to(torch.int32).view(torch.float32).clone()
        best_twoF[flagged] = float("nan")
        return {"tmpl": kept[:, 0], "bin": kept[:, 1], "twoF": kept[:, 2].view(torch.float32),
                "count": n, "best_twoF": best_twoF[:self.ntmpl],
                "best_bin": (best & 0xFFFFFFFF)[:self.ntmpl]}

    def run_profiled(self, out=None, stream=None):
        import torch
        dd = self.dd
        tf = out if out is not None else torch.empty((self.ntmpl, dd.n_bins), dtype=torch.float32,
                                                     device=dd.device)
        ms = (ctypes.c_float * 4)()
        cnt = (ctypes.c_int64 * 4)()
        _check(load_library().fstat_search_run_profiled(
            self.handle, ctypes.byref(dd.inputs), _ptr(self.templates), _ptr(tf), _ptr(self.ws),
            self.ws.numel(), _stream_ptr(stream), ms, cnt))
        return tf, {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNELS)}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fstat_search_destroy(self.handle)
            self.handle = None


class Batch:
    """Independent searches run as one captured graph (fstat_batch_*): each
    search keeps its own plan, data, templates, output and workspace; `lanes`
    concurrent branches.  run() returns the list of 2F outputs."""

    def __init__(self, searches, lanes=4):
        lib = load_library()
        self.searches = list(searches)
        arr = (ctypes.c_void_p * len(self.searches))(*[s.handle for s in self.searches])
        h = ctypes.c_void_p()
        _check(lib.fstat_batch_create(arr, len(self.searches), int(lanes), ctypes.byref(h)))
        self.handle = h

    def run(self, outs=None, stream=None):
        import torch
        n = len(self.searches)
        if outs is None:
            outs = [torch.empty((s.ntmpl, s.dd.n_bins), dtype=torch.float32, device=s.dd.device)
                    for s in self.searches]
        ins = (ctypes.POINTER(FstatInputs) * n)(*[ctypes.pointer(s.dd.inputs)
                                                  for s in self.searches])
        vp = ctypes.c_void_p
        tm = (vp * n)(*[_ptr(s.templates) for s in self.searches])
        tf = (vp * n)(*[_ptr(o) for o in outs])
        ws = (vp * n)(*[_ptr(s.ws) for s in self.searches])
        wb = (ctypes.c_size_t * n)(*[s.ws.numel() for s in self.searches])
        # the graph is launched on a stream of its own (a capture needs a
        # non-null stream), ordered after and before the caller's stream
        cur = torch.cuda.current_stream()
        if stream is None:
            if getattr(self, "stream", None) is None:
                self.stream = torch.cuda.Stream()
            st = self.stream
            st.wait_stream(cur)
        else:
            st = stream
        _check(load_library().fstat_batch_run(self.handle, ins, tm, tf, ws, wb, _stream_ptr(st)))
        if stream is None:
            cur.wait_stream(st)
        return outs

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fstat_batch_destroy(self.handle)
            self.handle = None
