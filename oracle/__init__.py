"""FP64 CPU oracle for Viola-Jones discrete AdaBoost -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path (the HIP library and its binding)
never imports, links or calls it; the two share no code.  The arithmetic lives
in ``vj_oracle.c`` (plain loops, FP64, sequential sums); this module only
marshals numpy arrays to it and sequences the steps of Section 2.3.

Parity status of each function (what pins it, see tests/test_oracle_pins.py):
  feature enumeration      printed counts of Section 2.2, closed form, brute force
  integral image, rect sum direct pixel sums (brute force)
  feature values           direct pixel sums over the rectangles
  best stump per feature   brute force over every integer threshold, both polarities
  round / update           Section 2.3 invariants (sum w = 1, T+ = T- = 1/2 at
                           round 1, previous stump has error exactly 1/2 under
                           the updated weights), threshold re-evaluation
  strong classifier        brute force of the Section 2.3 vote; log-base invariance
The dark/white shading of each feature type is a reading (Figure 3 is missing):
parity unpinned against the paper for the sign, pinned by the invariance of
every error under a global sign flip.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PLAIN_LIB_PATH = os.path.join(_HERE, "libvj_oracle.so")
SAN_LIB_PATH = os.path.join(_HERE, "libvj_oracle_san.so")
# VJB_ORACLE_SAN=1 loads the AddressSanitizer / UndefinedBehaviorSanitizer
# build (gcc's runtimes must then be preloaded into the interpreter)
SANITIZED = os.environ.get("VJB_ORACLE_SAN") == "1"
LIB_PATH = SAN_LIB_PATH if SANITIZED else PLAIN_LIB_PATH
SRC_PATH = os.path.join(_HERE, "vj_oracle.c")

TYPE_NAMES = ("3h", "3v", "2h", "2v", "4")
ALL_TYPES = 0x1F


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math); sanitize:
    the AddressSanitizer + UndefinedBehaviorSanitizer build instead."""
    path = SAN_LIB_PATH if sanitize else PLAIN_LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC_PATH):
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", SRC_PATH, "-o", tmp, "-lm"]
        if sanitize:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                        "-g"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


class _Stump(ctypes.Structure):
    _fields_ = [("err_pos", ctypes.c_double), ("err_neg", ctypes.c_double),
                ("err", ctypes.c_double), ("polarity", ctypes.c_int32),
                ("split", ctypes.c_int32), ("theta", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class _RoundRec(ctypes.Structure):
    _fields_ = [("feature", ctypes.c_int64), ("polarity", ctypes.c_int32),
                ("theta", ctypes.c_int32), ("split", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("err_raw", ctypes.c_double),
                ("err", ctypes.c_double), ("beta", ctypes.c_double),
                ("alpha", ctypes.c_double), ("t_pos", ctypes.c_double),
                ("t_neg", ctypes.c_double)]


STUMP_DTYPE = np.dtype([("err_pos", "<f8"), ("err_neg", "<f8"), ("err", "<f8"),
                        ("polarity", "<i4"), ("split", "<i4"), ("theta", "<i4"),
                        ("pad", "<i4")])
assert STUMP_DTYPE.itemsize == ctypes.sizeof(_Stump)

_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False, sanitize=SANITIZED)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.or_feature_count.restype = i64
        L.or_feature_count.argtypes = [i32, i32, i32]
        L.or_enumerate.restype = i64
        L.or_enumerate.argtypes = [i32, i32, i32, P]
        L.or_integral.argtypes = [P, i32, i32, P]
        L.or_rect_sum.restype = ctypes.c_int32
        L.or_rect_sum.argtypes = [P, i32, i32, i32, i32, i32]
        L.or_feature_value.restype = ctypes.c_int32
        L.or_feature_value.argtypes = [P, i32, P]
        L.or_integrals.argtypes = [P, i64, i32, i32, P, i32]
        L.or_feature_values.argtypes = [P, i64, i32, i32, P, i64, P, i32]
        L.or_sort_features.argtypes = [P, i64, i64, P, i32]
        L.or_best_stumps.argtypes = [P, P, P, P, i64, i64, P, i32]
        L.or_round.restype = i32
        L.or_round.argtypes = [P, P, P, P, i64, i64, dbl, P, ctypes.POINTER(_RoundRec), i32]
        L.or_init_weights.restype = i32
        L.or_init_weights.argtypes = [P, i64, P]
        L.or_strong_classify.argtypes = [P, P, P, P, i64, i64, P]
        L.or_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(lib().or_num_threads())


# ----------------------------------------------------------------- features
def feature_count(W: int, H: int, type_mask: int = ALL_TYPES) -> int:
    return int(lib().or_feature_count(W, H, type_mask))


def enumerate_features(W: int, H: int, type_mask: int = ALL_TYPES) -> np.ndarray:
    """int32 [F, 5] = (type, x, y, cw, ch) in the global feature order."""
    F = feature_count(W, H, type_mask)
    out = np.zeros((F, 5), np.int32)
    n = lib().or_enumerate(W, H, type_mask, _p(out))
    assert n == F
    return out


# ----------------------------------------------------------------- images
def integral(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.zeros((H + 1, W + 1), np.int32)
    lib().or_integral(_p(img), W, H, _p(out))
    return out


def integrals(images: np.ndarray, threads: int = 0) -> np.ndarray:
    images = np.ascontiguousarray(images, dtype=np.uint8)
    N, H, W = images.shape
    out = np.zeros((N, H + 1, W + 1), np.int32)
    lib().or_integrals(_p(images), N, W, H, _p(out), threads)
    return out


def rect_sum(ii: np.ndarray, x: int, y: int, w: int, h: int) -> int:
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    W = ii.shape[1] - 1
    return int(lib().or_rect_sum(_p(ii), W, x, y, w, h))


def feature_values(ii: np.ndarray, feats: np.ndarray, threads: int = 0) -> np.ndarray:
    """int32 [nf, N]: value of each feature on each window."""
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    feats = np.ascontiguousarray(feats, dtype=np.int32).reshape(-1, 5)
    N, H1, W1 = ii.shape
    out = np.zeros((feats.shape[0], N), np.int32)
    lib().or_feature_values(_p(ii), N, W1 - 1, H1 - 1, _p(feats), feats.shape[0], _p(out), threads)
    return out


def sort_features(vals: np.ndarray, threads: int = 0) -> np.ndarray:
    vals = np.ascontiguousarray(vals, dtype=np.int32)
    nf, N = vals.shape
    out = np.zeros((nf, N), np.int32)
    lib().or_sort_features(_p(vals), N, nf, _p(out), threads)
    return out


def best_stumps(vals, order, labels, w, threads: int = 0) -> np.ndarray:
    """Per-feature best stump (structured array with err_pos, err_neg, err,
    polarity, split, theta) under the given weights (used as given)."""
    vals = np.ascontiguousarray(vals, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    y = np.ascontiguousarray(labels, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float64)
    nf, N = vals.shape
    out = np.zeros(nf, STUMP_DTYPE)
    lib().or_best_stumps(_p(vals), _p(order), _p(y), _p(w), N, nf, _p(out), threads)
    return out


def init_weights(labels) -> np.ndarray:
    y = np.ascontiguousarray(labels, dtype=np.uint8)
    w = np.zeros(len(y), np.float64)
    if lib().or_init_weights(_p(y), len(y), _p(w)) != 0:
        raise ValueError("both classes must be present")
    return w


@dataclass
class RoundRecord:
    feature: int
    polarity: int
    theta: int
    split: int
    err_raw: float
    err: float
    beta: float
    alpha: float
    t_pos: float
    t_neg: float


def boost_round(vals, order, labels, w, eps_floor: float = 1e-10, threads: int = 0,
                scratch=None):
    """One round of Section 2.3 on prepared values/orders.  ``w`` (float64) is
    normalised and updated in place.  Returns (RoundRecord, per-feature stumps)."""
    vals = np.ascontiguousarray(vals, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    y = np.ascontiguousarray(labels, dtype=np.uint8)
    assert w.dtype == np.float64 and w.flags["C_CONTIGUOUS"]
    nf, N = vals.shape
    if scratch is None:
        scratch = np.zeros(nf, STUMP_DTYPE)
    rec = _RoundRec()
    rc = lib().or_round(_p(vals), _p(order), _p(y), _p(w), N, nf, eps_floor,
                        _p(scratch), ctypes.byref(rec), threads)
    if rc != 0:
        raise ValueError("weights sum to zero")
    r = RoundRecord(rec.feature, rec.polarity, rec.theta, rec.split, rec.err_raw,
                    rec.err, rec.beta, rec.alpha, rec.t_pos, rec.t_neg)
    return r, scratch


def strong_classify(fvals, polarity, theta, alpha) -> np.ndarray:
    """Section 2.3 strong classifier on precomputed feature values [T, N]."""
    fvals = np.ascontiguousarray(fvals, dtype=np.int32)
    T, N = fvals.shape
    pol = np.ascontiguousarray(polarity, dtype=np.int32)
    th = np.ascontiguousarray(theta, dtype=np.int32)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    out = np.zeros(N, np.uint8)
    lib().or_strong_classify(_p(fvals), _p(pol), _p(th), _p(al), T, N, _p(out))
    return out


class Trainer:
    """Sequences the oracle: integral images, values and orders once, then rounds."""

    def __init__(self, images, labels, type_mask: int = ALL_TYPES, threads: int = 0,
                 features=None):
        images = np.ascontiguousarray(images, dtype=np.uint8)
        self.N, self.H, self.W = images.shape
        self.labels = np.ascontiguousarray(labels, dtype=np.uint8)
        self.threads = threads
        self.feats = enumerate_features(self.W, self.H, type_mask) if features is None \
            else np.ascontiguousarray(features, dtype=np.int32)
        self.ii = integrals(images, threads)
        self.vals = feature_values(self.ii, self.feats, threads)
        self.order = sort_features(self.vals, threads)
        self.w = init_weights(self.labels)
        self.scratch = np.zeros(len(self.feats), STUMP_DTYPE)

    def round(self, eps_floor: float = 1e-10, weights=None):
        """One round; ``weights`` (if given) replace the current weights first
        (teacher forcing)."""
        if weights is not None:
            self.w = np.array(weights, dtype=np.float64, copy=True)
        rec, st = boost_round(self.vals, self.order, self.labels, self.w, eps_floor,
                              self.threads, self.scratch)
        return rec, st

    def train(self, rounds: int, eps_floor: float = 1e-10):
        out = []
        for _ in range(rounds):
            rec, _ = self.round(eps_floor)
            out.append(rec)
        return out
