"""Python binding of libcurvealign (MI355X / gfx950 closed-curve alignment).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/curvealign.h.  Tensors are torch
CUDA (HIP) tensors used as device memory; calls are enqueued on the current
torch stream unless a stream is given.

Result records (32 bytes each) are returned as a uint8 CUDA tensor of shape
[count, 32]; `unpack` turns them into named tensors or `to_numpy` into a
numpy structured array with fields shift, flags, theta, e0, err_est, gap.
"""
from __future__ import annotations

import ctypes
import os
import threading
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcurvealign.so")

RESULT_DTYPE = np.dtype([("shift", "<i4"), ("flags", "<u4"), ("theta", "<f8"),
                         ("e0", "<f8"), ("err_est", "<f4"), ("gap", "<f4")])
RESULT_BYTES = RESULT_DTYPE.itemsize

OK = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED_N = -2
ERR_HIP = -3
ERR_OOM = -4
ERR_NO_DEVICE = -5
ERR_INTERNAL = -6
ERR_TOO_LARGE = -7

FLAG_NEAR_TIE = 1 << 0
FLAG_RESCORED = 1 << 1
FLAG_CAND_CAPPED = 1 << 2
FLAG_DEGENERATE = 1 << 3
FLAG_NONFINITE = 1 << 4
FLAG_THETA_FP64 = 1 << 5
FLAG_UNSUPPORTED_N = 1 << 6
FLAG_CLOCKWISE = 1 << 7

PRECISION = {"fp32": 0, "split_bf16": 1, "fp64": 2}
RESCORE = {"top2": 0, "window": 1}
RESAMPLE = {"spline": 0, "linear": 1}
MAX_N = 4096
NOALLOC_SCRATCH_BYTES = 16 * 1024 * 1024 + 64 * 1024   # static scratch of align_all_pairs_noalloc
RESAMPLE_MAX_RAW = 32768   # raw vertices per curve accepted by resample_arclength

EXPORTED = ("ca_create", "ca_destroy", "ca_status_string", "ca_last_error", "ca_n_supported",
            "align_pair", "align_batch", "align_all_pairs", "align_all_pairs_noalloc", "resample_arclength",
            "to_initializer",
            "srv_transform", "ca_graph_begin", "ca_graph_end", "ca_graph_launch", "ca_graph_destroy", "ca_autotune", "ca_tune_get", "ca_tune_set", "ca_tune_save", "ca_tune_load")

# launch-tuning knobs (ca_autotune / ca_tune_*)
TUNE_KNOBS = {"team_grid": 0, "allpairs_cols": 1, "block_plan": 2, "block_grid": 3, "block_threads": 4}
# tuning cache shipped with the package, loaded by default_context when it
# matches the device; CURVEALIGN_TUNE_FILE names another file ("" = none)
TUNE_CACHE = os.path.join(_HERE, "tune_cache.json")


class CurveAlignError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"curvealign status {status}: {msg}")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rescore", ctypes.c_int32),
                ("theta_fp64", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libcurvealign.so (no fallback: a missing library is an error)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing; build it with "
                                  "`python -c 'import __graft_entry__ as g; g.build()'`")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
            L.ca_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_char_p]
            L.ca_destroy.argtypes = [vp]
            L.ca_status_string.argtypes = [i32]
            L.ca_status_string.restype = ctypes.c_char_p
            L.ca_last_error.argtypes = []
            L.ca_last_error.restype = ctypes.c_char_p
            L.ca_n_supported.argtypes = [i32]
            L.ca_n_supported.restype = i32
            L.align_pair.argtypes = [vp, vp, vp, i32, vp, vp, vp]
            L.align_batch.argtypes = [vp, vp, vp, vp, i32, i64, vp, vp, vp]
            L.align_all_pairs.argtypes = [vp, vp, i32, i32, vp, vp, vp]
            L.align_all_pairs_noalloc.argtypes = [vp, vp, i32, i32, vp, vp, vp]
            L.resample_arclength.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, i32, vp]
            L.to_initializer.argtypes = [vp, vp, i32, vp, i64, vp, vp, vp]
            L.srv_transform.argtypes = [vp, vp, vp, i32, i64, vp, vp]
            L.ca_graph_begin.argtypes = [vp, ctypes.POINTER(vp)]
            L.ca_graph_end.argtypes = [vp, ctypes.POINTER(vp)]
            L.ca_graph_launch.argtypes = [vp, vp]
            L.ca_graph_destroy.argtypes = [vp]
            pi32 = ctypes.POINTER(i32)
            L.ca_autotune.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_float), vp]
            L.ca_tune_get.argtypes = [vp, i32, i32, pi32, pi32]
            L.ca_tune_set.argtypes = [vp, i32, i32, pi32, i32]
            L.ca_tune_save.argtypes = [vp, ctypes.c_char_p]
            L.ca_tune_load.argtypes = [vp, ctypes.c_char_p, pi32]
            for name in ("ca_create", "ca_destroy", "align_pair", "align_batch",
                         "align_all_pairs", "align_all_pairs_noalloc", "resample_arclength", "to_initializer", "srv_transform",
                         "ca_graph_begin", "ca_graph_end", "ca_graph_launch", "ca_graph_destroy",
                         "ca_autotune", "ca_tune_get", "ca_tune_set", "ca_tune_save", "ca_tune_load"):
                getattr(L, name).restype = i32
            _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        L = lib()
        raise CurveAlignError(status, f"{L.ca_status_string(status).decode()}: "
                                      f"{L.ca_last_error().decode()}")


def n_supported(n: int) -> bool:
    return bool(lib().ca_n_supported(int(n)))


class Context:
    """Owns the library context (plans, twiddle tables, workspace) on one device."""

    def __init__(self, device: int = 0, tune_file: str | None = None):
        self.device = int(device)
        h = ctypes.c_void_p()
        path = None if tune_file is None else os.fsencode(tune_file)
        _check(lib().ca_create(ctypes.byref(h), self.device, path))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().ca_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def default_context(device: int | None = None) -> Context:
    """The per-device context of this process, created on first use with the
    tuning cache (CURVEALIGN_TUNE_FILE, else the packaged one) loaded; a cache
    that cannot be read leaves the default launch choices (with a warning)."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        ctx = Context(dev)
        ctx.tune_applied = 0
        path = os.environ.get("CURVEALIGN_TUNE_FILE", TUNE_CACHE)
        if path and os.path.exists(path):
            try:
                ctx.tune_applied = tune_load(path, ctx=ctx)
            except CurveAlignError as e:      # unreadable cache: the defaults stay in force
                warnings.warn(f"tuning cache {path} not loaded ({e}); using default launch choices")
        _contexts[dev] = ctx
    return _contexts[dev]


class Graph:
    """A HIP graph the library recorded (ca_graph_begin / ca_graph_end):
    `launch(stream=None)` replays it on a torch stream (current by default)."""

    def __init__(self, handle, ctx):
        self.handle = handle
        self.ctx = ctx        # the context must outlive the graph

    def launch(self, stream=None):
        _check(lib().ca_graph_launch(self.handle, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().ca_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(fn, *, ctx=None, device=None):
    """Record the library calls fn(stream) makes on the capture stream into a
    library-owned HIP graph.  fn receives a torch ExternalStream to pass as the
    `stream=` argument of every call it makes."""
    import torch
    ctx = ctx or default_context(device)
    torch.cuda.synchronize()
    h = ctypes.c_void_p()
    _check(lib().ca_graph_begin(ctx.handle, ctypes.byref(h)))
    stream = torch.cuda.ExternalStream(h.value, device=torch.device("cuda", ctx.device))
    g = ctypes.c_void_p()
    try:
        fn(stream)
    finally:
        st = lib().ca_graph_end(ctx.handle, ctypes.byref(g))
    _check(st)
    return Graph(g, ctx)


def _knob(knob) -> int:
    if knob not in TUNE_KNOBS:
        raise ValueError(f"knob must be one of {sorted(TUNE_KNOBS)}")
    return TUNE_KNOBS[knob]


def autotune(knob: str, key: int, *, stream=None, ctx=None) -> float:
    """Time every candidate of (knob, key) on a synthetic batch, install the
    fastest; returns its milliseconds per launch."""
    ctx = ctx or default_context()
    ms = ctypes.c_float()
    _check(lib().ca_autotune(ctx.handle, _knob(knob), int(key), ctypes.byref(ms), _stream_ptr(stream)))
    return float(ms.value)


def tune_get(knob: str, key: int, *, ctx=None) -> list[int]:
    ctx = ctx or default_context()
    vals = (ctypes.c_int32 * 16)()
    cnt = ctypes.c_int32(16)
    _check(lib().ca_tune_get(ctx.handle, _knob(knob), int(key), vals, ctypes.byref(cnt)))
    return [int(vals[i]) for i in range(cnt.value)]


def tune_set(knob: str, key: int, values, *, ctx=None):
    ctx = ctx or default_context()
    vals = [int(v) for v in (values if hasattr(values, "__len__") else [values])]
    arr = (ctypes.c_int32 * max(1, len(vals)))(*vals)
    _check(lib().ca_tune_set(ctx.handle, _knob(knob), int(key), arr, len(vals)))


def tune_save(path: str, *, ctx=None):
    ctx = ctx or default_context()
    _check(lib().ca_tune_save(ctx.handle, os.fsencode(path)))


def tune_load(path: str, *, ctx=None) -> int:
    """Install the entries of a tuning file; returns how many applied (0 for
    a file written for another device)."""
    ctx = ctx or default_context()
    applied = ctypes.c_int32(0)
    _check(lib().ca_tune_load(ctx.handle, os.fsencode(path), ctypes.byref(applied)))
    return int(applied.value)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _options(precision: str, rescore: str, theta_fp64: bool) -> _Options:
    if precision not in PRECISION:
        raise ValueError(f"precision must be one of {sorted(PRECISION)}")
    if rescore not in RESCORE:
        raise ValueError(f"rescore must be one of {sorted(RESCORE)}")
    return _Options(PRECISION[precision], RESCORE[rescore], 1 if theta_fp64 else 0, 0)


def _require(t, what, dtypes, ndim=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must live on a GPU device")
    if t.dtype not in dtypes:
        raise TypeError(f"{what} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{what} must have {ndim} dims")


def empty_results(count: int, device):
    import torch
    return torch.empty((int(count), RESULT_BYTES), dtype=torch.uint8, device=device)


def unpack(res):
    """Named views of a [count, 32] uint8 result tensor (no copies)."""
    import torch
    w32 = res.view(torch.int32).view(-1, 8)
    f32 = res.view(torch.float32).view(-1, 8)
    f64 = res.view(torch.float64).view(-1, 4)
    return {"shift": w32[:, 0], "flags": w32[:, 1], "theta": f64[:, 1], "e0": f64[:, 2],
            "err_est": f32[:, 6], "gap": f32[:, 7]}


def to_numpy(res) -> np.ndarray:
    return res.cpu().numpy().view(RESULT_DTYPE).reshape(-1)


def align_pair(z1, z2, *, precision="fp32", rescore="top2", theta_fp64=False, out=None,
               stream=None, ctx=None):
    """Optimal start shift, rotation and e0 for one pair of n-node curves."""
    import torch
    dt = (torch.complex128,) if precision == "fp64" else (torch.complex64,)
    _require(z1, "z1", dt, 1)
    _require(z2, "z2", dt, 1)
    if z1.shape != z2.shape:
        raise ValueError("z1 and z2 must have the same length")
    ctx = ctx or default_context(z1.device.index)
    out = empty_results(1, z1.device) if out is None else out
    opt = _options(precision, rescore, theta_fp64)
    _check(lib().align_pair(ctx.handle, z1.data_ptr(), z2.data_ptr(), z1.shape[0],
                            out.data_ptr(), ctypes.byref(opt), _stream_ptr(stream)))
    return out


def align_batch(z1, z2, offsets=None, *, precision="fp32", rescore="top2", theta_fp64=False,
                out=None, stream=None, ctx=None):
    """Uniform batch: z1, z2 of shape [B, n].  Ragged batch: z1, z2 flat [total]
    with int64 `offsets` [B+1] (device tensor)."""
    import torch
    dt = (torch.complex128,) if precision == "fp64" else (torch.complex64,)
    _require(z1, "z1", dt)
    _require(z2, "z2", dt)
    if z1.shape != z2.shape:
        raise ValueError("z1 and z2 must have the same shape")
    if offsets is None:
        if z1.dim() != 2:
            raise ValueError("uniform batches are [B, n]")
        B, n = z1.shape
        off_ptr = None
    else:
        _require(offsets, "offsets", (torch.int64,), 1)
        B, n = offsets.shape[0] - 1, 0
        off_ptr = offsets.data_ptr()
    ctx = ctx or default_context(z1.device.index)
    out = empty_results(B, z1.device) if out is None else out
    opt = _options(precision, rescore, theta_fp64)
    _check(lib().align_batch(ctx.handle, z1.data_ptr(), z2.data_ptr(), off_ptr, n, B,
                             out.data_ptr(), ctypes.byref(opt), _stream_ptr(stream)))
    return out


def align_all_pairs(curves, *, rescore="top2", theta_fp64=False, out=None, stream=None, ctx=None):
    """All i<j pairs of a gallery [m, n]; results in row-major upper-triangle order."""
    import torch
    _require(curves, "curves", (torch.complex64,), 2)
    m, n = curves.shape
    ctx = ctx or default_context(curves.device.index)
    out = empty_results(m * (m - 1) // 2, curves.device) if out is None else out
    opt = _options("fp32", rescore, theta_fp64)
    _check(lib().align_all_pairs(ctx.handle, curves.data_ptr(), m, n, out.data_ptr(),
                                 ctypes.byref(opt), _stream_ptr(stream)))
    return out


def noalloc_scratch_bytes(m: int, n: int) -> int:
    """Static scratch align_all_pairs_noalloc needs for an m x n gallery."""
    return (m * n * 8 + 255) // 256 * 256 + m * 8


def align_all_pairs_noalloc(curves, out, *, rescore="top2", theta_fp64=False, stream=None, ctx=None):
    """align_all_pairs through the entry point that allocates nothing: the
    caller passes the [m(m-1)/2, 32] uint8 output; the spectra live in the
    library's static per-device scratch (calls on one device must not overlap)."""
    import torch
    _require(curves, "curves", (torch.complex64,), 2)
    _require(out, "out", (torch.uint8,), 2)
    m, n = curves.shape
    if out.shape[0] < m * (m - 1) // 2 or out.shape[1] != RESULT_BYTES:
        raise ValueError("out must be [m(m-1)/2, 32] uint8")
    ctx = ctx or default_context(curves.device.index)
    opt = _options("fp32", rescore, theta_fp64)
    _check(lib().align_all_pairs_noalloc(ctx.handle, curves.data_ptr(), m, n, out.data_ptr(),
                                         ctypes.byref(opt), _stream_ptr(stream)))
    return out


def to_initializer(results, n=None, offsets=None, *, stream=None, ctx=None):
    """Alignment records -> the paper's (t0*, R*) for an elastic solver.

    `results` is the uint8 [count, 32] tensor from align_*; give the uniform
    node count `n` or the ragged `offsets` used for the alignment.  Returns
    (t0 FP64 [count], R FP64 [count, 2, 2]).
    """
    import torch
    _require(results, "results", (torch.uint8,), 2)
    count = results.shape[0]
    if (n is None) == (offsets is None):
        raise ValueError("give exactly one of n and offsets")
    if offsets is not None:
        _require(offsets, "offsets", (torch.int64,), 1)
        if offsets.shape[0] != count + 1:
            raise ValueError("offsets must have count + 1 entries")
    ctx = ctx or default_context(results.device.index)
    t0 = torch.empty(count, dtype=torch.float64, device=results.device)
    rot = torch.empty(count, 2, 2, dtype=torch.float64, device=results.device)
    _check(lib().to_initializer(ctx.handle, results.data_ptr(), 0 if n is None else int(n),
                                None if offsets is None else offsets.data_ptr(), count,
                                t0.data_ptr(), rot.data_ptr(), _stream_ptr(stream)))
    return t0, rot


def srv_transform(curves, offsets=None, *, out=None, stream=None, ctx=None):
    """Square-root-velocity values q_k of closed polygons (section 3).

    Uniform: curves complex64 [count, n].  Ragged: curves flat complex64 with
    int64 `offsets` [count+1].  Returns q with the layout of `curves`."""
    import torch
    _require(curves, "curves", (torch.complex64,))
    if offsets is None:
        if curves.dim() != 2:
            raise ValueError("uniform curves are [count, n]")
        count, n, off_ptr = curves.shape[0], curves.shape[1], None
    else:
        _require(offsets, "offsets", (torch.int64,), 1)
        if curves.dim() != 1:
            raise ValueError("ragged curves are flat")
        count, n, off_ptr = offsets.shape[0] - 1, 0, offsets.data_ptr()
    ctx = ctx or default_context(curves.device.index)
    out = torch.empty_like(curves) if out is None else out
    _check(lib().srv_transform(ctx.handle, curves.data_ptr(), off_ptr, n, count, out.data_ptr(),
                               _stream_ptr(stream)))
    return out


def resample_arclength(raw, raw_offsets, out_offsets, *, mode="spline", with_norms=True,
                       with_flags=True, out=None, stream=None, ctx=None):
    """Raw polygons (complex64 flat, int64 offsets [C+1]) -> uniform arc-length
    nodes (complex64 flat, laid out by out_offsets).  Returns (nodes, norms, flags)."""
    import torch
    _require(raw, "raw", (torch.complex64,), 1)
    _require(raw_offsets, "raw_offsets", (torch.int64,), 1)
    _require(out_offsets, "out_offsets", (torch.int64,), 1)
    if mode not in RESAMPLE:
        raise ValueError(f"mode must be one of {sorted(RESAMPLE)}")
    C = raw_offsets.shape[0] - 1
    if out_offsets.shape[0] != C + 1:
        raise ValueError("raw_offsets and out_offsets must have the same length")
    total = int(out_offsets[-1].item()) if out is None else out.shape[0]
    ctx = ctx or default_context(raw.device.index)
    out = torch.empty(total, dtype=torch.complex64, device=raw.device) if out is None else out
    norms = torch.empty(C, dtype=torch.float64, device=raw.device) if with_norms else None
    flags = torch.empty(C, dtype=torch.int32, device=raw.device) if with_flags else None
    _check(lib().resample_arclength(ctx.handle, raw.data_ptr(), raw_offsets.data_ptr(), C,
                                    out_offsets.data_ptr(), out.data_ptr(),
                                    norms.data_ptr() if norms is not None else None,
                                    flags.data_ptr() if flags is not None else None,
                                    RESAMPLE[mode], _stream_ptr(stream)))
    return out, norms, flags
