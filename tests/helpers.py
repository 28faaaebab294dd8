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


# ------------------------------------------------------------ the weight update
# Section 2.3 step 4 is FP64 on the GPU in every precision mode.  Two checks
# hold it there:
#  * given the GPU's own stump and beta, the updated weights follow from the
#    round's input weights by a handful of FP64 operations on either side
#    (a product, two normalisations), so they agree to a few units of
#    2^-53: UPDATE_RTOL.  An update done in FP32 would miss by ~2^-24.
#  * against the oracle's updated weights, where both picked the same stump
#    but their betas differ (the scan's error differs within its tolerance):
#    w_i <- w_i b_i / Z with b_i = beta for correctly classified windows, 1
#    otherwise.  A change of ln beta moves ln w_i by the same amount for
#    every correct window and by nothing for the others, and normalising
#    subtracts one common amount, so the spread of ln(w_gpu / w_oracle) over
#    the windows grows by at most |ln(beta_gpu / beta_oracle)| per round;
#    both vectors sum to one, so every |ln(w_gpu / w_oracle)| is at most that
#    spread (weight_rtol).
UPDATE_RTOL = 1e-14


def updated_weights(vals_j: np.ndarray, labels: np.ndarray, w_norm: np.ndarray, polarity: int, theta: int,
                    beta: float) -> np.ndarray:
    """w_i * beta^(1 - e_i), normalised, for the stump (polarity, theta) on
    feature values vals_j (Section 2.3 step 4 and the next round's step 1)."""
    h = (polarity * vals_j.astype(np.int64) < polarity * int(theta)).astype(np.int64)
    correct = h == labels.astype(np.int64)
    w = np.where(correct, w_norm * beta, w_norm)
    return w / w.sum()


def weight_rtol(betas_gpu, betas_oracle) -> float:
    """Bound on |w_gpu / w_oracle - 1| after the rounds whose betas are given
    (same stumps on both sides), plus UPDATE_RTOL per round for rounding."""
    bg = np.atleast_1d(np.asarray(betas_gpu, dtype=np.float64))
    bo = np.atleast_1d(np.asarray(betas_oracle, dtype=np.float64))
    spread = float(np.sum(np.abs(np.log(bg / bo))))
    return float(np.expm1(spread)) + UPDATE_RTOL * len(bg)


def assert_weights(w_gpu: np.ndarray, w_ref: np.ndarray, rtol: float, what: str = ""):
    """|w_gpu / w_ref - 1| <= rtol where w_ref > 0; exactly 0 where w_ref is 0."""
    assert np.all(np.isfinite(w_gpu)), what
    z = w_ref == 0
    assert np.all(w_gpu[z] == 0), (what, "a zero weight became nonzero", int(np.argmax(w_gpu[z] != 0)))
    r = np.zeros_like(w_ref)
    r[~z] = np.abs(w_gpu[~z] / w_ref[~z] - 1.0)
    assert float(r.max()) <= rtol, (what, float(r.max()), rtol, int(np.argmax(r)))
