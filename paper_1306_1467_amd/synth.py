"""Seeded synthetic training windows for Viola-Jones AdaBoost workloads.

This module only draws inputs; it holds none of the boosting arithmetic and is
shared by the tests, the oracle harness and the benchmark so that every side
sees the same bytes for the same seed.

The paper trains on the Viola-Jones face set (4,916 faces + 7,960 non-faces of
24x24 grey windows, Section 2.2); that set is not available here, so these
generators stand in for it with the same window size, grey-level uint8 pixels
and comparable class counts.  Nothing of the face set is reproduced.

Recipe (all randomness from ``numpy.random.Generator(PCG64(SeedSequence(seed)))``):

* template(r0, c): a 24x24 piecewise-constant face-like pattern -- background
  115, a forehead block and two cheek blocks at 115 + c/2, a horizontal dark
  band of four rows starting at row r0 at 115 - c/2 -- blurred with a Gaussian
  of sigma 1 (half-sample symmetric boundary), then nearest-neighbour resampled
  to the window size s.
* positive window: template + N(0, 15) per pixel, rounded half-to-even,
  clipped to [0, 255].
* negative window: iid uniform bytes, blurred with sigma ~ U[0, 2] (no blur
  when sigma < 0.05), rounded half-to-even, clipped.
* samples are ordered positives first.
"""
from __future__ import annotations

from dataclasses import dataclass
import math
import os

import numpy as np

BACKGROUND = 115.0


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))


def _gauss_kernel(sigma: float) -> np.ndarray:
    radius = int(4.0 * sigma + 0.5)
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _reflect_index(n: int, radius: int) -> np.ndarray:
    """Indices of a half-sample symmetric extension ``d c b a | a b c d | d c b a``."""
    idx = np.arange(-radius, n + radius)
    period = 2 * n
    idx = np.mod(idx, period)
    return np.where(idx < n, idx, period - 1 - idx)


def gaussian_blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of one 2-D float image (truncated at 4 sigma)."""
    if sigma < 0.05:
        return img.astype(np.float64, copy=True)
    k = _gauss_kernel(sigma)
    r = (len(k) - 1) // 2
    out = img.astype(np.float64)
    for axis in (0, 1):
        n = out.shape[axis]
        ext = np.take(out, _reflect_index(n, r), axis=axis)
        acc = np.zeros_like(out)
        for t in range(len(k)):
            acc += k[t] * np.take(ext, np.arange(t, t + n), axis=axis)
        out = acc
    return out


def _blur_taps(cur: np.ndarray, k: np.ndarray, lo: int, r: int, rmax: int) -> np.ndarray:
    """Separable blur of a [m, h, w] stack by per-image kernels k [m, 2 rmax + 1]
    that are zero outside taps rmax - r .. rmax + r (lo = rmax - r)."""
    for axis in (1, 2):
        n = cur.shape[axis]
        ext = np.take(cur, _reflect_index(n, r), axis=axis)
        acc = np.zeros_like(cur)
        for t in range(2 * r + 1):
            sl = np.take(ext, np.arange(t, t + n), axis=axis)
            acc += k[:, lo + t][:, None, None] * sl
        cur = acc
    return cur


def gaussian_blur_batch(imgs: np.ndarray, sigmas: np.ndarray) -> np.ndarray:
    """Blur each image of a [n, h, w] stack with its own sigma (vectorised).

    Images whose sigma is below 0.05 are returned unblurred.  Each image's
    kernel has taps |t| <= round(4 sigma), normalised over a common row of
    2 rmax + 1 taps (zero beyond its own radius); the images are blurred in
    groups of equal radius, on several threads, adding only the nonzero taps
    in tap order, which gives the same values as adding every tap of the
    common row (the skipped terms are exact zeros).
    """
    imgs = imgs.astype(np.float64)
    out = imgs.copy()
    sig = np.asarray(sigmas, dtype=np.float64)
    sel = np.nonzero(sig >= 0.05)[0]
    if len(sel) == 0:
        return out
    rmax = int(4.0 * sig[sel].max() + 0.5)
    taps = np.arange(-rmax, rmax + 1, dtype=np.float64)
    s = sig[sel][:, None]
    radius = np.floor(4.0 * s + 0.5)
    k = np.exp(-0.5 * (taps[None, :] / s) ** 2) * (np.abs(taps[None, :]) <= radius)
    k /= k.sum(axis=1, keepdims=True)
    rad = radius[:, 0].astype(np.int64)
    work = []
    for r in np.unique(rad):
        idx = np.nonzero(rad == r)[0]
        for c in range(0, len(idx), 2048):
            work.append((int(r), idx[c:c + 2048]))

    def run(item):
        r, idx = item
        return idx, _blur_taps(imgs[sel[idx]], k[idx], rmax - r, r, rmax)

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        for idx, res in ex.map(run, work):
            out[sel[idx]] = res
    return out


def template(r0: int, contrast: float, size: int = 24) -> np.ndarray:
    """Face-like template, float64 [size, size], before noise."""
    t = np.full((24, 24), BACKGROUND, dtype=np.float64)
    hi = BACKGROUND + contrast / 2.0
    lo = BACKGROUND - contrast / 2.0
    t[2:max(2, r0 - 1), 4:20] = hi                 # forehead
    t[r0:r0 + 4, 2:22] = lo                        # dark band (eyes)
    t[r0 + 5:r0 + 11, 3:9] = hi                    # left cheek
    t[r0 + 5:r0 + 11, 15:21] = hi                  # right cheek
    t = gaussian_blur(t, 1.0)
    if size != 24:
        src = (np.arange(size) * 24) // size
        t = t[np.ix_(src, src)]
    return t


def _to_u8(x: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def make_job(seed, n_pos: int, n_neg: int, size: int = 24, r0: int = 7,
             contrast: float = 110.0):
    """One seeded training set: (images uint8 [N, size, size], labels uint8 [N]).

    Positives come first.
    """
    rng = _rng(seed)
    tpl = template(r0, contrast, size)
    pos = _to_u8(tpl[None] + rng.normal(0.0, 15.0, size=(n_pos, size, size)))
    raw = rng.integers(0, 256, size=(n_neg, size, size)).astype(np.float64)
    sig = rng.uniform(0.0, 2.0, size=n_neg)
    neg = _to_u8(gaussian_blur_batch(raw, sig))
    images = np.concatenate([pos, neg], axis=0)
    labels = np.concatenate([np.ones(n_pos, np.uint8), np.zeros(n_neg, np.uint8)])
    return images, labels


def _log_uniform(rng: np.random.Generator, a: float, b: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(a), math.log(b)))))


@dataclass
class JobSpec:
    seed: tuple
    n_pos: int
    n_neg: int
    size: int
    r0: int
    contrast: float
    rounds: int

    @property
    def n(self) -> int:
        return self.n_pos + self.n_neg

    def make(self):
        return make_job(self.seed, self.n_pos, self.n_neg, self.size, self.r0, self.contrast)


WORKLOADS = ("tiny", "faces15k", "batch32", "batch64")


def workload_jobs(name: str):
    """Job specs of the named workloads.

    tiny:     128 + 128 windows of 24x24, r0 = 7, contrast 110, 5 rounds.
    faces15k: 5,000 + 10,000 windows of 24x24, same template, 200 rounds
              (the size of the paper's face training set).
    batch32:  32 jobs, 24x24, positives log-uniform in [500, 5000], negatives
              twice the positives, r0 ~ U{5..12}, contrast ~ U[60, 140],
              50 rounds.
    batch64:  64 jobs, window 16/20/24/28, positives log-uniform in
              [1000, 8000], negatives log-uniform in [2000, 20000],
              r0 ~ U{5..12}, contrast ~ U[60, 140], 100 rounds.
    """
    if name == "tiny":
        return [JobSpec((0,), 128, 128, 24, 7, 110.0, 5)]
    if name == "faces15k":
        return [JobSpec((1,), 5000, 10000, 24, 7, 110.0, 200)]
    if name == "batch32":
        jobs = []
        for j in range(32):
            rng = _rng((3, j, 0))
            l = _log_uniform(rng, 500, 5000)
            r0 = int(rng.integers(5, 13))
            c = float(rng.uniform(60, 140))
            jobs.append(JobSpec((3, j), l, 2 * l, 24, r0, c, 50))
        return jobs
    if name == "batch64":
        jobs = []
        for j in range(64):
            rng = _rng((4, j, 0))
            s = int(rng.choice([16, 20, 24, 28]))
            l = _log_uniform(rng, 1000, 8000)
            m = _log_uniform(rng, 2000, 20000)
            r0 = int(rng.integers(5, 13))
            c = float(rng.uniform(60, 140))
            jobs.append(JobSpec((4, j), l, m, s, r0, c, 100))
        return jobs
    raise ValueError(f"unknown workload {name!r}")


def small_job(seed, n: int, size: int, levels: int = 4, pos_frac: float = 0.5):
    """Tiny window sets with a small pixel alphabet, so that feature values tie often.

    Returns (images uint8 [n, size, size], labels uint8 [n]); labels are drawn,
    not sorted, with at least one sample of each class.
    """
    rng = _rng(seed)
    alphabet = np.linspace(0, 255, levels).round().astype(np.uint8)
    images = alphabet[rng.integers(0, levels, size=(n, size, size))]
    labels = (rng.uniform(size=n) < pos_frac).astype(np.uint8)
    if labels.sum() == 0:
        labels[0] = 1
    if labels.sum() == n:
        labels[-1] = 0
    return images, labels


def random_weights(seed, n: int, lo_exp: float = -20.0, hi_exp: float = 0.0):
    """Positive weights log-uniform over [10**lo_exp, 10**hi_exp] (not normalised)."""
    rng = _rng(seed)
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size=n)
