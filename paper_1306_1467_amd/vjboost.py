"""Thin ctypes binding of libvjboost (include/vjboost.h).

Argument marshalling only: every step of the training path runs in the HIP
library.  PyTorch provides device memory (workspace, inputs, outputs) and the
stream.  Importing this module does not need a GPU; loading the library does
need the built ``libvjboost.so`` and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VJBOOST_LIB selects another build of the library (the sanitizer build)
LIB_PATH = os.environ.get("VJBOOST_LIB") or os.path.join(HERE, "libvjboost.so")

BOOST_OK = 0
BOOST_E_INVALID = -1
BOOST_E_NOMEM = -2
BOOST_E_DEVICE = -3
BOOST_E_DEGENERATE = -4

BOOST_PREC_FP32 = 0
BOOST_PREC_FP32_KAHAN = 1
BOOST_PREC_FP64 = 2
BOOST_PREC_FP32_WIDE = 3
PRECISIONS = {"fp32": BOOST_PREC_FP32, "fp32_kahan": BOOST_PREC_FP32_KAHAN,
              "fp64": BOOST_PREC_FP64, "fp32_wide": BOOST_PREC_FP32_WIDE}

BOOST_ON_PERFECT_CLAMP = 0
BOOST_ON_PERFECT_STOP = 1
BOOST_FLAG_TIMING = 1
BOOST_FLAG_NO_GRAPH = 2
BOOST_SCHEDULE_AUTO = -1
BOOST_ALL_TYPES = 0x1F


class FeatureSet(ctypes.Structure):
    _fields_ = [("window_w", ctypes.c_int32), ("window_h", ctypes.c_int32),
                ("type_mask", ctypes.c_uint32)]


class Feature(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("x", ctypes.c_int32), ("y", ctypes.c_int32),
                ("cell_w", ctypes.c_int32), ("cell_h", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("on_perfect", ctypes.c_int32),
                ("eps_floor", ctypes.c_double), ("schedule_id", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class Stump(ctypes.Structure):
    _fields_ = [("feature", ctypes.c_int64), ("type", ctypes.c_int32), ("x", ctypes.c_int32),
                ("y", ctypes.c_int32), ("cell_w", ctypes.c_int32), ("cell_h", ctypes.c_int32),
                ("polarity", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("split_rank", ctypes.c_int32), ("round", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("error_raw", ctypes.c_double), ("error", ctypes.c_double),
                ("beta", ctypes.c_double), ("alpha", ctypes.c_double)]


class Job(ctypes.Structure):
    _fields_ = [("d_images", ctypes.c_void_p), ("d_labels", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("fs", FeatureSet)]


STUMP_DTYPE = np.dtype([("feature", "<i8"), ("type", "<i4"), ("x", "<i4"), ("y", "<i4"),
                        ("cell_w", "<i4"), ("cell_h", "<i4"), ("polarity", "<i4"),
                        ("threshold", "<i4"), ("split_rank", "<i4"), ("round", "<i4"),
                        ("pad", "<i4"), ("error_raw", "<f8"), ("error", "<f8"),
                        ("beta", "<f8"), ("alpha", "<f8")])
assert STUMP_DTYPE.itemsize == ctypes.sizeof(Stump) == 80

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "boost_version": (ctypes.c_int, []),
    "boost_last_error": (ctypes.c_char_p, []),
    "boost_options_default": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "boost_feature_count": (ctypes.c_int64, [ctypes.POINTER(FeatureSet)]),
    "boost_feature_desc": (ctypes.c_int, [ctypes.POINTER(FeatureSet), ctypes.c_int64, ctypes.POINTER(Feature)]),
    "boost_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.POINTER(FeatureSet), ctypes.POINTER(Options)]),
    "boost_schedule_count": (ctypes.c_int, [ctypes.c_int32]),
    "boost_tune_cache_clear": (None, []),
    "boost_get_schedule": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "boost_probe_stream": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "boost_init": (ctypes.c_int, [ctypes.POINTER(_P), _P, _P, ctypes.c_int64, ctypes.POINTER(FeatureSet),
                                  ctypes.POINTER(Options), _P, ctypes.c_size_t]),
    "boost_extend_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int64]),
    "boost_extend": (ctypes.c_int, [ctypes.POINTER(_P), _P, _P, _P, ctypes.c_int64, _P, ctypes.c_size_t]),
    "boost_extend_merged": (ctypes.c_int, [_P]),
    "boost_round": (ctypes.c_int, [_P, ctypes.POINTER(Stump), _P]),
    "boost_train": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "boost_get_weights": (ctypes.c_int, [_P, _P]),
    "boost_set_weights": (ctypes.c_int, [_P, _P]),
    "boost_rounds_done": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "boost_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "boost_reset_timing": (ctypes.c_int, [_P]),
    "boost_get_feature_values": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P]),
    "boost_get_integral": (ctypes.c_int, [_P, _P]),
    "boost_get_sorted": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "boost_classify_train": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    "boost_classify_train_curve": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    "boost_classify_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "boost_classify": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32,
                                      _P, _P, _P, _P, _P, ctypes.c_size_t]),
    "boost_classify_noalloc_max_windows": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "boost_classify_noalloc": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                              ctypes.c_int32, _P, _P, _P, _P]),
    "boost_destroy": (None, [_P]),
    "boost_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, _P, ctypes.POINTER(Options)]),
    "boost_batch_init": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.POINTER(Options), _P,
                                        ctypes.c_size_t]),
    "boost_batch_round": (ctypes.c_int, [_P, _P]),
    "boost_batch_train": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "boost_batch_get_weights": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "boost_batch_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "boost_batch_get_schedule": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32)]),
    "boost_batch_destroy": (None, [_P]),
}

_lib = None


def lib():
    """Load libvjboost.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1306_1467_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class BoostError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def last_error() -> str:
    s = lib().boost_last_error()
    return s.decode() if s else ""


def _check(rc: int):
    if rc != BOOST_OK:
        raise BoostError(rc, last_error())


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def feature_set(window_w: int, window_h: int | None = None, type_mask: int = BOOST_ALL_TYPES) -> FeatureSet:
    return FeatureSet(window_w, window_h if window_h is not None else window_w, type_mask)


def options(precision="fp32_wide", on_perfect: int = BOOST_ON_PERFECT_CLAMP, eps_floor: float = 1e-10,
            schedule_id: int = 0, flags: int = 0, stream: int | None = None) -> Options:
    o = Options()
    _check(lib().boost_options_default(ctypes.byref(o)))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.on_perfect = on_perfect
    o.eps_floor = eps_floor
    o.schedule_id = schedule_id
    o.flags = flags
    o.stream = stream
    return o


# ------------------------------------------------------------------ host-only calls
def boost_feature_count(fs: FeatureSet) -> int:
    return int(lib().boost_feature_count(ctypes.byref(fs)))


def boost_feature_desc(fs: FeatureSet, j: int):
    f = Feature()
    _check(lib().boost_feature_desc(ctypes.byref(fs), j, ctypes.byref(f)))
    return (f.type, f.x, f.y, f.cell_w, f.cell_h)


def boost_workspace_bytes(n: int, fs: FeatureSet, opts: Options) -> int:
    return int(lib().boost_workspace_bytes(n, ctypes.byref(fs), ctypes.byref(opts)))


def boost_schedule_count(precision: int = BOOST_PREC_FP32_WIDE) -> int:
    return int(lib().boost_schedule_count(precision))


# ------------------------------------------------------------------ device calls
def boost_init(d_images, d_labels, n: int, fs: FeatureSet, opts: Options, d_workspace, workspace_bytes: int):
    h = ctypes.c_void_p()
    _check(lib().boost_init(ctypes.byref(h), _ptr(d_images), _ptr(d_labels), n, ctypes.byref(fs),
                            ctypes.byref(opts), _ptr(d_workspace), workspace_bytes))
    return h


def boost_extend_workspace_bytes(ctx, m: int) -> int:
    return int(lib().boost_extend_workspace_bytes(ctx, m))


def boost_extend(ctx, d_images, d_labels, m: int, d_workspace, workspace_bytes: int):
    h = ctypes.c_void_p()
    _check(lib().boost_extend(ctypes.byref(h), ctx, _ptr(d_images), _ptr(d_labels), m, _ptr(d_workspace),
                              workspace_bytes))
    return h


def boost_extend_merged(ctx) -> bool:
    rc = lib().boost_extend_merged(ctx)
    _check(min(rc, 0))
    return rc == 1


def boost_round(ctx, want_record: bool = True, d_feature_err=None):
    rec = Stump() if want_record else None
    _check(lib().boost_round(ctx, ctypes.byref(rec) if rec is not None else None, _ptr(d_feature_err)))
    return rec


def boost_train(ctx, rounds: int, want_records: bool = True):
    out = np.zeros(rounds, STUMP_DTYPE) if want_records else None
    _check(lib().boost_train(ctx, rounds, out.ctypes.data if out is not None else None))
    return out


def boost_get_weights(ctx, d_w):
    _check(lib().boost_get_weights(ctx, _ptr(d_w)))


def boost_set_weights(ctx, d_w):
    _check(lib().boost_set_weights(ctx, _ptr(d_w)))


def boost_rounds_done(ctx) -> int:
    r = ctypes.c_int32()
    _check(lib().boost_rounds_done(ctx, ctypes.byref(r)))
    return int(r.value)


def boost_get_timing(ctx):
    out = (ctypes.c_double * 4)()
    _check(lib().boost_get_timing(ctx, out))
    return list(out)


def boost_reset_timing(ctx):
    _check(lib().boost_reset_timing(ctx))


def boost_get_schedule(ctx):
    """(schedule in use, per-schedule tuning times in ms or -1 where not timed)."""
    cap = boost_schedule_count()
    ms = (ctypes.c_double * cap)()
    rc = lib().boost_get_schedule(ctx, ctypes.cast(ms, _P), cap)
    _check(min(rc, 0))
    return int(rc), list(ms)


def boost_probe_stream(ctx, reps: int = 5) -> float:
    """Fastest of `reps` launches (ms) of a kernel that reads every key with
    the scan's access pattern and no arithmetic."""
    ms = ctypes.c_double(0.0)
    _check(lib().boost_probe_stream(ctx, reps, ctypes.byref(ms)))
    return float(ms.value)


def boost_tune_cache_clear():
    lib().boost_tune_cache_clear()


def boost_get_feature_values(ctx, j0: int, nf: int, d_out):
    _check(lib().boost_get_feature_values(ctx, j0, nf, _ptr(d_out)))


def boost_get_integral(ctx, d_out):
    _check(lib().boost_get_integral(ctx, _ptr(d_out)))


def boost_get_sorted(ctx, j0: int, nf: int, d_order, d_run_end):
    _check(lib().boost_get_sorted(ctx, j0, nf, _ptr(d_order), _ptr(d_run_end)))


def boost_classify_train(ctx, stumps: np.ndarray, d_out, d_score=None):
    stumps = np.ascontiguousarray(stumps, dtype=STUMP_DTYPE)
    _check(lib().boost_classify_train(ctx, stumps.ctypes.data if len(stumps) else None, len(stumps),
                                      _ptr(d_out), _ptr(d_score)))


def boost_classify_train_curve(ctx, stumps: np.ndarray, d_curve):
    stumps = np.ascontiguousarray(stumps, dtype=STUMP_DTYPE)
    _check(lib().boost_classify_train_curve(ctx, stumps.ctypes.data if len(stumps) else None, len(stumps),
                                            _ptr(d_curve)))


def boost_classify_workspace_bytes(n: int, window_w: int, window_h: int) -> int:
    return int(lib().boost_classify_workspace_bytes(n, window_w, window_h))


def boost_classify(d_images, n: int, window_w: int, window_h: int, d_labels, stumps: np.ndarray, d_out, d_score,
                   d_curve, stream, d_workspace, workspace_bytes: int):
    stumps = np.ascontiguousarray(stumps, dtype=STUMP_DTYPE)
    _check(lib().boost_classify(_ptr(d_images), n, window_w, window_h, _ptr(d_labels),
                                stumps.ctypes.data if len(stumps) else None, len(stumps), _ptr(d_out), _ptr(d_score),
                                _ptr(d_curve), stream, _ptr(d_workspace), workspace_bytes))


def boost_classify_noalloc_max_windows(window_w: int, window_h: int) -> int:
    return int(lib().boost_classify_noalloc_max_windows(window_w, window_h))


def boost_classify_noalloc(d_images, n: int, window_w: int, window_h: int, d_labels, stumps: np.ndarray, d_out,
                           d_score, d_curve, stream):
    stumps = np.ascontiguousarray(stumps, dtype=STUMP_DTYPE)
    _check(lib().boost_classify_noalloc(_ptr(d_images), n, window_w, window_h, _ptr(d_labels),
                                        stumps.ctypes.data if len(stumps) else None, len(stumps), _ptr(d_out),
                                        _ptr(d_score), _ptr(d_curve), stream))


def classify(images, stumps, labels=None, device: str = "cuda:0"):
    """The strong classifier of the records `stumps` on windows `images`
    (uint8 [N, H, W], host or device): (decisions uint8 [N], scores float64
    [N], error curve int32 [T] or None) as torch tensors on the device.  The
    curve needs labels: entry t - 1 counts the windows the first t stumps
    misclassify."""
    torch = _torch()
    dev = torch.device(device)
    img = torch.as_tensor(images).to(dev).contiguous()
    if img.dtype != torch.uint8 or img.dim() != 3:
        raise ValueError("images must be uint8 [N, H, W]")
    n, h, w = (int(v) for v in img.shape)
    lab = None if labels is None else torch.as_tensor(labels).to(dev).contiguous()
    stumps = np.ascontiguousarray(stumps, dtype=STUMP_DTYPE)
    T = len(stumps)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    score = torch.empty(n, dtype=torch.float64, device=dev)
    curve = torch.empty(max(T, 1), dtype=torch.int32, device=dev) if lab is not None else None
    ws_bytes = boost_classify_workspace_bytes(n, w, h)
    if ws_bytes == 0:
        raise BoostError(BOOST_E_INVALID, "invalid window set")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    boost_classify(img, n, w, h, lab, stumps, out, score, curve, stream.cuda_stream, ws, ws_bytes)
    return out, score, (curve[:T] if curve is not None else None)


def boost_destroy(ctx):
    if ctx is not None:
        lib().boost_destroy(ctx)


def boost_batch_workspace_bytes(jobs_arr, opts: Options) -> int:
    return int(lib().boost_batch_workspace_bytes(len(jobs_arr), ctypes.cast(jobs_arr, ctypes.c_void_p),
                                                 ctypes.byref(opts)))


def boost_batch_init(jobs_arr, opts: Options, d_workspace, workspace_bytes: int):
    h = ctypes.c_void_p()
    _check(lib().boost_batch_init(ctypes.byref(h), len(jobs_arr), ctypes.cast(jobs_arr, ctypes.c_void_p),
                                  ctypes.byref(opts), _ptr(d_workspace), workspace_bytes))
    return h


def boost_batch_round(b, n_jobs: int, want_records: bool = True):
    out = np.zeros(n_jobs, STUMP_DTYPE) if want_records else None
    _check(lib().boost_batch_round(b, out.ctypes.data if out is not None else None))
    return out


def boost_batch_train(b, rounds: int, n_jobs: int, want_records: bool = True):
    out = np.zeros((rounds, n_jobs), STUMP_DTYPE) if want_records else None
    _check(lib().boost_batch_train(b, rounds, out.ctypes.data if out is not None else None))
    return out


def boost_batch_get_weights(b, job: int, d_w):
    _check(lib().boost_batch_get_weights(b, job, _ptr(d_w)))


def boost_batch_get_timing(b):
    out = (ctypes.c_double * 4)()
    _check(lib().boost_batch_get_timing(b, out))
    return list(out)


def boost_batch_get_schedule(b, key_format: int):
    """(schedule id or -1 when absent, segments per workgroup) of the scan
    launch for key format 0 (14-bit keys) or 1 (15-bit keys)."""
    sched = ctypes.c_int32(0)
    spw = ctypes.c_int32(0)
    _check(lib().boost_batch_get_schedule(b, key_format, ctypes.byref(sched), ctypes.byref(spw)))
    return int(sched.value), int(spw.value)


def boost_batch_destroy(b):
    if b is not None:
        lib().boost_batch_destroy(b)


# ------------------------------------------------------------------ convenience owners
def _torch():
    import torch
    return torch


class Trainer:
    """Owns one boosting context: torch-allocated inputs and workspace, a torch
    stream for the library's work (default priority)."""

    def __init__(self, images, labels, type_mask: int = BOOST_ALL_TYPES, precision="fp32_wide",
                 on_perfect: int = BOOST_ON_PERFECT_CLAMP, eps_floor: float = 1e-10,
                 schedule_id: int = 0, flags: int = 0, device: str = "cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        img = torch.as_tensor(images)
        lab = torch.as_tensor(labels)
        if img.dtype != torch.uint8 or lab.dtype != torch.uint8 or img.dim() != 3:
            raise ValueError("images must be uint8 [N, H, W] and labels uint8 [N]")
        self.n, self.h, self.w = (int(v) for v in img.shape)
        self.images = img.to(self.device).contiguous()
        self.labels = lab.to(self.device).contiguous()
        self.stream = torch.cuda.Stream(device=self.device)
        self.fs = feature_set(self.w, self.h, type_mask)
        self.opts = options(precision, on_perfect, eps_floor, schedule_id, flags, self.stream.cuda_stream)
        self.F = boost_feature_count(self.fs)
        self.ws_bytes = boost_workspace_bytes(self.n, self.fs, self.opts)
        if self.ws_bytes == 0:
            raise BoostError(BOOST_E_INVALID, last_error())
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        self.ctx = boost_init(self.images, self.labels, self.n, self.fs, self.opts, self.workspace, self.ws_bytes)
        self.init_s = time.perf_counter() - t0    # boost_init (it synchronises)

    def extend(self, images, labels):
        """A new Trainer over this trainer's windows followed by `images` /
        `labels` (boost_extend: the old windows' order is reused)."""
        torch = _torch()
        img = torch.as_tensor(images)
        lab = torch.as_tensor(labels)
        if img.dtype != torch.uint8 or lab.dtype != torch.uint8 or img.dim() != 3 or \
                tuple(img.shape[1:]) != (self.h, self.w):
            raise ValueError("images must be uint8 [M, H, W] of this trainer's window size, labels uint8 [M]")
        new = Trainer.__new__(Trainer)
        new.device = self.device
        m = int(img.shape[0])
        new.n, new.h, new.w = self.n + m, self.h, self.w
        new.images = img.to(self.device).contiguous()
        new.labels = lab.to(self.device).contiguous()
        new.stream = self.stream
        new.fs, new.opts, new.F = self.fs, self.opts, self.F
        new.ws_bytes = boost_extend_workspace_bytes(self.ctx, m)
        if new.ws_bytes == 0:
            raise BoostError(BOOST_E_INVALID, last_error())
        new.workspace = torch.empty(new.ws_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        new.ctx = boost_extend(self.ctx, new.images, new.labels, m, new.workspace, new.ws_bytes)
        new.init_s = time.perf_counter() - t0     # boost_extend (it synchronises)
        return new

    def merged(self) -> bool:
        return boost_extend_merged(self.ctx)

    # every device output is allocated here and filled on the library's stream
    def _sync(self):
        self.stream.synchronize()

    def round(self, feature_err: bool = False):
        torch = _torch()
        ferr = torch.empty((self.F, 2), dtype=torch.float64, device=self.device) if feature_err else None
        rec = boost_round(self.ctx, True, ferr)
        self._sync()
        return (rec, ferr) if feature_err else rec

    def train(self, rounds: int, want_records: bool = True):
        out = boost_train(self.ctx, rounds, want_records)
        return out

    def weights(self):
        torch = _torch()
        w = torch.empty(self.n, dtype=torch.float64, device=self.device)
        boost_get_weights(self.ctx, w)
        self._sync()
        return w

    def set_weights(self, w):
        torch = _torch()
        wt = torch.as_tensor(w, dtype=torch.float64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        boost_set_weights(self.ctx, wt)

    def feature_values(self, j0: int = 0, nf: int | None = None):
        torch = _torch()
        nf = self.F - j0 if nf is None else nf
        out = torch.empty((nf, self.n), dtype=torch.int32, device=self.device)
        boost_get_feature_values(self.ctx, j0, nf, out)
        self._sync()
        return out

    def integral(self):
        torch = _torch()
        out = torch.empty((self.n, self.h + 1, self.w + 1), dtype=torch.int32, device=self.device)
        boost_get_integral(self.ctx, out)
        self._sync()
        return out

    def sorted(self, j0: int, nf: int):
        torch = _torch()
        order = torch.empty((nf, self.n), dtype=torch.int32, device=self.device)
        flags = torch.empty((nf, self.n), dtype=torch.uint8, device=self.device)
        boost_get_sorted(self.ctx, j0, nf, order, flags)
        self._sync()
        return order, flags

    def classify(self, stumps):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.uint8, device=self.device)
        score = torch.empty(self.n, dtype=torch.float64, device=self.device)
        boost_classify_train(self.ctx, stumps, out, score)
        self._sync()
        return out, score

    def error_curve(self, stumps):
        """Training-error curve: entry t - 1 = training windows misclassified by the first t stumps."""
        torch = _torch()
        curve = torch.empty(max(len(stumps), 1), dtype=torch.int32, device=self.device)
        boost_classify_train_curve(self.ctx, stumps, curve)
        self._sync()
        return curve[:len(stumps)]

    def timing(self):
        return boost_get_timing(self.ctx)

    def rounds_done(self):
        return boost_rounds_done(self.ctx)

    def schedule(self):
        return boost_get_schedule(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            boost_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchTrainer:
    """Owns a batch of independent jobs advanced together (one scan launch and
    one update launch per round for all jobs)."""

    def __init__(self, datasets, type_mask: int = BOOST_ALL_TYPES, precision="fp32_wide",
                 on_perfect: int = BOOST_ON_PERFECT_CLAMP, eps_floor: float = 1e-10,
                 schedule_id: int = 0, flags: int = 0, device: str = "cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        self.inputs = []
        arr = (Job * len(datasets))()
        self.sizes = []
        for k, (images, labels) in enumerate(datasets):
            img = torch.as_tensor(images).to(self.device).contiguous()
            lab = torch.as_tensor(labels).to(self.device).contiguous()
            if img.dtype != torch.uint8 or lab.dtype != torch.uint8 or img.dim() != 3:
                raise ValueError("images must be uint8 [N, H, W] and labels uint8 [N]")
            n, h, w = (int(v) for v in img.shape)
            self.inputs.append((img, lab))
            self.sizes.append((n, h, w))
            arr[k] = Job(img.data_ptr(), lab.data_ptr(), n, feature_set(w, h, type_mask))
        self.jobs = arr
        self.n_jobs = len(datasets)
        self.stream = torch.cuda.Stream(device=self.device)
        self.opts = options(precision, on_perfect, eps_floor, schedule_id, flags, self.stream.cuda_stream)
        self.ws_bytes = boost_batch_workspace_bytes(arr, self.opts)
        if self.ws_bytes == 0:
            raise BoostError(BOOST_E_INVALID, last_error())
        t0 = time.perf_counter()
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.alloc_s = time.perf_counter() - t0   # the caller's workspace allocation
        t0 = time.perf_counter()
        self.ctx = boost_batch_init(arr, self.opts, self.workspace, self.ws_bytes)
        self.init_s = time.perf_counter() - t0    # boost_batch_init (it synchronises)

    def sync(self):
        self.stream.synchronize()

    def round(self):
        return boost_batch_round(self.ctx, self.n_jobs, True)

    def train(self, rounds: int, want_records: bool = True):
        return boost_batch_train(self.ctx, rounds, self.n_jobs, want_records)

    def weights(self, job: int):
        torch = _torch()
        w = torch.empty(self.sizes[job][0], dtype=torch.float64, device=self.device)
        boost_batch_get_weights(self.ctx, job, w)
        self.sync()
        return w

    def timing(self):
        return boost_batch_get_timing(self.ctx)

    def schedule(self):
        return [boost_batch_get_schedule(self.ctx, k) for k in (0, 1)]

    def close(self):
        if getattr(self, "ctx", None) is not None:
            boost_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
