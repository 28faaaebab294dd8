"""Shared helpers of the parity tests: tolerances and stump comparison rules."""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def err_tolerance(ref: np.ndarray, n: int, precision: str, keys_per_lane: int = 8) -> np.ndarray:
    """Allowed |gpu - oracle| per feature error.

    The oracle's own FP64 prefix sums carry at most ~2n u64 absolute error
    (weights sum to 1), so every bound has that floor.
      fp64, fp32_wide, fp32_kahan: 1e-6 relative + floor.  The compensated
        mode evaluates each candidate as s + c in FP64 (exact for two floats)
        and its two-sum carries the prefix to about u32^2, so, as with FP64
        sums of the FP32 weights, the error left is the FP32 rounding of each
        weight: at most 2^-24 relative on every error.
      fp32: recursive FP32 summation over a lane segment and the 64-lane scan:
        (keys_per_lane + 64) u32 absolute (plain FP32 meets no relative bound).
    """
    ref = np.abs(np.asarray(ref, dtype=np.float64))
    floor = 4.0 * n * U64
    if precision in ("fp64", "fp32_wide", "fp32_kahan"):
        return 1e-6 * ref + floor
    return np.full_like(ref, 2.0 * (keys_per_lane + 64) * U32 + floor)


def stump_error(vals_j: np.ndarray, labels: np.ndarray, w: np.ndarray, polarity: int, theta: int) -> float:
    """Weighted error of h = [p f < p theta] under w (Section 2.3 definition)."""
    h = (polarity * vals_j.astype(np.int64) < polarity * int(theta)).astype(np.int64)
    return float(np.sum(w[h != labels.astype(np.int64)]))


def check_stump(gpu, ost, orec, vals, labels, w_norm, n, precision):
    """Stump identity where the oracle's top two features are separated by more
    than the tolerance; otherwise the GPU's stump must be an equally good one.

    gpu: Stump record; ost: oracle per-feature stumps; orec: oracle round record;
    vals: oracle values [F, n] (caller order); w_norm: normalised weights of the round.
    """
    errs = ost["err"]
    best = float(errs[orec.feature])
    tol = float(err_tolerance(np.array([best]), n, precision)[0])
    # the GPU's stump re-evaluated by the definition
    e_gpu = stump_error(vals[gpu.feature], labels, w_norm, gpu.polarity, gpu.threshold)
    assert abs(e_gpu - best) <= tol, (gpu.feature, gpu.polarity, gpu.threshold, e_gpu, best)
    assert abs(gpu.error_raw - best) <= tol, (gpu.error_raw, best)
    order = np.argsort(errs, kind="stable")
    gap = float(errs[order[1]] - errs[order[0]]) if len(errs) > 1 else np.inf
    if gap > 2 * tol:
        assert gpu.feature == orec.feature
        assert gpu.polarity == orec.polarity
        # the threshold is unique when no other split of this feature ties
        if gpu.threshold != orec.theta:
            e2 = stump_error(vals[gpu.feature], labels, w_norm, gpu.polarity, gpu.threshold)
            assert abs(e2 - best) <= tol
