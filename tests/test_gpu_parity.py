"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes: the 24x24 / 256-window workload (all 162,336 features, every value and
every per-feature error compared), small windows with ragged sizes and heavy
ties, and edge cases.  The full 15,000-window workload is covered by sampled
features in test_gpu_fullsize.py.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1306_1467_amd import synth
from tests.helpers import UPDATE_RTOL, assert_weights, check_stump, err_tolerance, updated_weights, weight_rtol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny():
    spec = synth.workload_jobs("tiny")[0]
    images, labels = spec.make()
    say("building oracle for 24x24 x 256")
    otr = oracle.Trainer(images, labels)
    return images, labels, otr


def _trainer(images, labels, **kw):
    return vb.Trainer(torch.from_numpy(np.ascontiguousarray(images)),
                      torch.from_numpy(np.ascontiguousarray(labels)), **kw)


def test_integral_and_values_exact(tiny):
    images, labels, otr = tiny
    say("tiny: integral images + all feature values")
    tr = _trainer(images, labels)
    ii = tr.integral().cpu().numpy()
    assert (ii == otr.ii).all()
    vals = tr.feature_values().cpu().numpy()
    assert vals.shape == otr.vals.shape
    assert (vals == otr.vals).all()
    tr.close()


def test_sorted_keys(tiny):
    images, labels, otr = tiny
    say("tiny: sorted keys of all features")
    tr = _trainer(images, labels)
    F, n = otr.vals.shape
    step = 20000
    for j0 in range(0, F, step):
        nf = min(step, F - j0)
        order, flags = tr.sorted(j0, nf)
        order = order.cpu().numpy()
        flags = flags.cpu().numpy().astype(bool)
        assert (np.sort(order, axis=1) == np.arange(n)[None, :]).all()   # a permutation
        v = np.take_along_axis(otr.vals[j0:j0 + nf], order, axis=1)
        assert (np.diff(v, axis=1) >= 0).all()                           # ascending
        ends = np.ones_like(flags)
        ends[:, :-1] = v[:, 1:] != v[:, :-1]
        assert (flags == ends).all()                                      # run ends
    tr.close()


@pytest.mark.parametrize("precision", ["fp32_wide", "fp64", "fp32_kahan", "fp32"])
def test_rounds_teacher_forced(tiny, precision):
    """Per round: the oracle's weights go to both sides; every feature's error
    for both polarities, the stump, beta, alpha and the updated weights."""
    images, labels, otr = tiny
    say(f"tiny: 5 teacher-forced rounds, {precision}")
    tr = _trainer(images, labels, precision=precision)
    n = len(labels)
    w = oracle.init_weights(labels)
    for t in range(5):
        wn = w / w.sum()
        tr.set_weights(wn)
        rec, ferr = tr.round(feature_err=True)
        ferr = ferr.cpu().numpy()
        otr.w = w.copy()
        orec, ost = otr.round()
        tol_p = err_tolerance(ost["err_pos"], n, precision)
        tol_n = err_tolerance(ost["err_neg"], n, precision)
        dp = np.abs(ferr[:, 0] - ost["err_pos"])
        dn = np.abs(ferr[:, 1] - ost["err_neg"])
        assert (dp <= tol_p).all(), (t, precision, dp.max(), int(np.argmax(dp - tol_p)))
        assert (dn <= tol_n).all(), (t, precision, dn.max(), int(np.argmax(dn - tol_n)))
        check_stump(rec, ost, orec, otr.vals, labels, wn, n, precision)
        assert abs(rec.beta - rec.error / (1 - rec.error)) <= 1e-15 * max(1.0, rec.beta)
        # the FP64 update of Section 2.3 step 4, from the GPU's own stump and beta
        w_gpu = tr.weights().cpu().numpy()
        assert_weights(w_gpu, updated_weights(otr.vals[rec.feature], labels, wn, rec.polarity, rec.threshold,
                                              rec.beta), UPDATE_RTOL, f"update {precision} {t}")
        if rec.feature == orec.feature and rec.polarity == orec.polarity and rec.threshold == orec.theta:
            assert_weights(w_gpu, otr.w / otr.w.sum(), weight_rtol(rec.beta, orec.beta), f"oracle {precision} {t}")
        w = otr.w.copy()
    tr.close()


def _dyadic_weights(seed, n):
    """Integer weights 1..1000 scaled by 2^-m with a sum of exactly 1: every
    normalised weight, FP32 table entry and prefix sum (multiples of 2^-m, at
    most 1 in magnitude, m <= 24) is exact in every precision."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 1001, size=n).astype(np.int64)
    m = int(np.ceil(np.log2(k.sum())))
    k[int(rng.integers(0, n))] += (1 << m) - int(k.sum())
    assert k.sum() == 1 << m and m <= 24 and (k > 0).all()
    return k.astype(np.float64) / float(1 << m)


@pytest.mark.parametrize("precision", ["fp32_wide", "fp64", "fp32_kahan", "fp32"])
def test_exact_arithmetic_dyadic_weights(tiny, precision):
    """With weights on a coarse dyadic grid no operation rounds, on either
    side: every feature's errors, the stump and its error equal the oracle's
    bit for bit, in every precision."""
    images, labels, otr = tiny
    cases = [(images, labels, otr, 31)]
    ti, tl = synth.small_job((205, 1), 300, 8, 4)
    cases.append((ti, tl, oracle.Trainer(ti, tl), 32))
    for images_c, labels_c, otr_c, seed in cases:
        say(f"exact dyadic weights, {precision}, n = {len(labels_c)}")
        w = _dyadic_weights(seed, len(labels_c))
        tr = _trainer(images_c, labels_c, precision=precision)
        tr.set_weights(w)
        rec, ferr = tr.round(feature_err=True)
        ferr = ferr.cpu().numpy()
        orec, ost = otr_c.round(weights=w)
        assert np.array_equal(ferr[:, 0], ost["err_pos"])
        assert np.array_equal(ferr[:, 1], ost["err_neg"])
        assert (rec.feature, rec.polarity, rec.threshold, rec.split_rank) == \
            (orec.feature, orec.polarity, orec.theta, orec.split)
        assert rec.error_raw == orec.err_raw
        # equal errors give equal betas; the FP64 update then agrees to rounding
        assert rec.beta == orec.beta and abs(rec.alpha - orec.alpha) <= 1e-15 * max(1.0, abs(orec.alpha))
        assert_weights(tr.weights().cpu().numpy(), otr_c.w / otr_c.w.sum(), UPDATE_RTOL, f"dyadic {precision}")
        tr.close()


def test_free_running_matches_oracle(tiny):
    images, labels, _ = tiny
    say("tiny: 5 free-running rounds fp32_wide")
    tr = _trainer(images, labels, precision="fp32_wide")
    otr = oracle.Trainer(images, labels)
    n = len(labels)
    recs = tr.train(5)
    for t in range(5):
        wn = otr.w / otr.w.sum()
        orec, ost = otr.round()
        g = recs[t]
        assert g["round"] == t
        e = float(g["error_raw"])
        assert abs(e - orec.err_raw) <= err_tolerance(np.array([orec.err_raw]), n, "fp32_wide")[0]
        from tests.helpers import stump_error
        assert abs(stump_error(otr.vals[g["feature"]], labels, wn, int(g["polarity"]), int(g["threshold"]))
                   - orec.err_raw) <= 1e-9
    assert tr.rounds_done() == 5
    tr.close()


def _tiny(seed, n, size, levels, pos_frac=0.5):
    images, labels = synth.small_job((200, seed), n, size, levels, pos_frac)
    return images, labels


@pytest.mark.parametrize("seed,n,size,levels", [
    (0, 2, 4, 2),         # minimum n
    (1, 37, 6, 3),        # ragged n, one partial key unit
    (2, 511, 8, 4),       # several lanes, ties everywhere
    (3, 513, 8, 256),     # just over 512 keys
    (4, 1000, 5, 2),      # binary pixels
    (5, 4099, 6, 16),     # q >= 1 with remainder lanes
])
def test_small_windows_all_features(seed, n, size, levels):
    images, labels = _tiny(seed, n, size, levels)
    say(f"tiny: seed={seed} n={n} size={size} levels={levels}")
    otr = oracle.Trainer(images, labels)
    for precision in ("fp32_wide", "fp64"):
        tr = _trainer(images, labels, precision=precision)
        assert (tr.feature_values().cpu().numpy() == otr.vals).all()
        w = synth.random_weights((201, seed), n, -6, 0)
        for t in range(3):
            wn = w / w.sum()
            tr.set_weights(wn)
            rec, ferr = tr.round(feature_err=True)
            ferr = ferr.cpu().numpy()
            otr.w = w.copy()
            orec, ost = otr.round()
            assert (np.abs(ferr[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, precision)).all()
            assert (np.abs(ferr[:, 1] - ost["err_neg"]) <= err_tolerance(ost["err_neg"], n, precision)).all()
            check_stump(rec, ost, orec, otr.vals, labels, wn, n, precision)
            w = otr.w.copy()
        tr.close()


def test_window_sizes_and_type_masks():
    for size, mask in [(16, 0x1F), (20, 0x05), (28, 0x10), (32, 0x08), (3, 0x1F), (1, 0x1F)]:
        say(f"window {size} mask {mask:#x}")
        images, labels = synth.make_job((300, size), 60, 70, size=size, r0=7, contrast=40.0) if size >= 16 \
            else _tiny(size, 90, size, 256)
        otr = oracle.Trainer(images, labels, type_mask=mask)
        if len(otr.feats) == 0:
            continue
        tr = _trainer(images, labels, type_mask=mask)
        assert tr.F == len(otr.feats)
        assert (tr.feature_values().cpu().numpy() == otr.vals).all()
        rec, ferr = tr.round(feature_err=True)
        orec, ost = otr.round()
        n = len(labels)
        assert (np.abs(ferr.cpu().numpy()[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
        tr.close()


def test_shuffled_labels_caller_order():
    # positives not first in the caller's order: outputs stay in caller order
    images, labels = synth.make_job((400,), 50, 80, size=12, r0=4, contrast=50.0)
    perm = np.random.default_rng(0).permutation(len(labels))
    images, labels = images[perm], labels[perm]
    say("shuffled caller order")
    otr = oracle.Trainer(images, labels)
    tr = _trainer(images, labels)
    assert (tr.integral().cpu().numpy() == otr.ii).all()
    assert (tr.feature_values().cpu().numpy() == otr.vals).all()
    w0 = tr.weights().cpu().numpy()
    ow = otr.w / otr.w.sum()
    assert np.allclose(w0, ow, rtol=1e-15)
    rec = tr.round()
    orec, ost = otr.round()
    check_stump(rec, ost, orec, otr.vals, labels, ow, len(labels), "fp32_wide")
    w1 = tr.weights().cpu().numpy()
    assert_weights(w1, updated_weights(otr.vals[rec.feature], labels, ow, rec.polarity, rec.threshold, rec.beta),
                   UPDATE_RTOL, "shuffled")
    if rec.feature == orec.feature and rec.threshold == orec.theta and rec.polarity == orec.polarity:
        assert_weights(w1, otr.w / otr.w.sum(), weight_rtol(rec.beta, orec.beta), "shuffled oracle")
    tr.close()


def test_perfect_split_clamp_and_stop():
    n = 64
    images = np.zeros((n, 4, 4), np.uint8)
    labels = np.zeros(n, np.uint8)
    labels[::3] = 1
    images[labels == 1, :, 2:] = 200
    say("perfect split: clamp and stop")
    tr = _trainer(images, labels, on_perfect=vb.BOOST_ON_PERFECT_CLAMP)
    rec = tr.round()
    assert rec.error_raw == 0.0 and rec.error == 1e-10
    w = tr.weights().cpu().numpy()
    assert np.isfinite(w).all() and abs(w.sum() - 1) < 1e-12
    tr.close()
    tr = _trainer(images, labels, on_perfect=vb.BOOST_ON_PERFECT_STOP)
    with pytest.raises(vb.BoostError) as ei:
        tr.round()
    assert ei.value.code == vb.BOOST_E_DEGENERATE
    w_before = tr.weights().cpu().numpy()
    recs = None
    with pytest.raises(vb.BoostError):
        recs = tr.train(3)
    assert np.array_equal(tr.weights().cpu().numpy(), w_before)
    assert tr.rounds_done() == 1
    tr.close()


def test_invalid_inputs_rejected():
    say("invalid inputs")
    images, labels = _tiny(9, 20, 6, 4)
    bad = labels.copy()
    bad[3] = 2
    with pytest.raises(vb.BoostError) as ei:
        _trainer(images, bad)
    assert ei.value.code == vb.BOOST_E_INVALID
    with pytest.raises(vb.BoostError):
        _trainer(images, np.ones_like(labels))
    tr = _trainer(images, labels)
    for w in (np.full(20, np.nan), -np.ones(20), np.zeros(20), np.full(20, np.inf)):
        with pytest.raises(vb.BoostError):
            tr.set_weights(w)
    # the previous weights survive a rejected update
    assert abs(tr.weights().cpu().numpy().sum() - 1.0) < 1e-12
    tr.close()


def test_graph_and_direct_agree():
    images, labels = synth.make_job((500,), 300, 500, size=16, r0=5, contrast=30.0)
    say("graph vs direct vs timing launches")
    a = _trainer(images, labels)
    b = _trainer(images, labels, flags=vb.BOOST_FLAG_NO_GRAPH)
    c = _trainer(images, labels, flags=vb.BOOST_FLAG_TIMING)
    ra, rb, rc = a.train(12), b.train(12), c.train(12)
    assert ra.tobytes() == rb.tobytes() == rc.tobytes()
    assert np.array_equal(a.weights().cpu().numpy(), b.weights().cpu().numpy())
    t = c.timing()
    assert t[2] == 12 and t[0] > 0 and t[1] > 0
    # per-round calls give the same records as one train call
    d = _trainer(images, labels)
    rd = [d.round() for _ in range(12)]
    assert all(rd[i].feature == ra[i]["feature"] and rd[i].error_raw == ra[i]["error_raw"] for i in range(12))
    for x in (a, b, c, d):
        x.close()


def test_schedules_agree():
    images, labels = synth.make_job((600,), 700, 900, size=20, r0=6, contrast=35.0)
    say("all scan schedules give identical results")
    ref = None
    for s in range(vb.boost_schedule_count()):
        tr = _trainer(images, labels, schedule_id=s)
        r = tr.train(4)
        w = tr.weights().cpu().numpy()
        if ref is None:
            ref = (r, w)
        else:
            assert r.tobytes() == ref[0].tobytes()
            assert np.array_equal(w, ref[1])
        tr.close()


# Schedules 9 and 10 scan with rotating loads (512 and 1024 threads): lanes
# scan a whole number of 4-unit batches per feature (padding units add zero
# and hold no split) and the loads run one batch ahead across feature
# boundaries.  Shapes: one key unit per lane or less, exactly one batch, one
# unit past it, many batches with remainder lanes, feature counts far below
# one workgroup step (empty groups and waves), and 15-bit keys.
ROTATING = 9
ROTATING_SCHEDULES = (9, 10)


@pytest.mark.parametrize("seed,n,size,levels", [
    (0, 2, 4, 2),         # per = 1: the fill stream moves to the next feature at once
    (1, 37, 6, 3),        # per = 1, ragged units
    (2, 512, 8, 4),       # per = 4: exactly one batch
    (3, 513, 8, 256),     # per = 5: one unit past a batch
    (4, 4099, 6, 16),     # many batches, remainder lanes
    (5, 300, 3, 4),       # 3x3 windows: fewer features than one workgroup step
    (6, 16500, 5, 64),    # 15-bit keys
])
def test_rotating_loads_match_batched(seed, n, size, levels):
    images, labels = _tiny(seed, n, size, levels)
    say(f"rotating loads: seed={seed} n={n} size={size}")
    assert vb.boost_schedule_count() > max(ROTATING_SCHEDULES)
    precisions = ["fp32_wide", "fp32_kahan", "fp32"] + (["fp64"] if n <= 20000 else [])
    for precision in precisions:
        ref = _trainer(images, labels, precision=precision, schedule_id=0)
        a = ref.train(5)
        wa = ref.weights().cpu().numpy()
        ref.close()
        for sched in ROTATING_SCHEDULES:
            tr = _trainer(images, labels, precision=precision, schedule_id=sched)
            b = tr.train(5)
            wb = tr.weights().cpu().numpy()
            tr.close()
            assert b.tobytes() == a.tobytes(), (precision, sched)
            assert np.array_equal(wb, wa), (precision, sched)


def test_rotating_loads_against_oracle(tiny):
    images, labels, otr = tiny
    say("tiny: rotating loads, per-feature errors against the oracle")
    n = len(labels)
    tr = _trainer(images, labels, schedule_id=ROTATING)
    w = synth.random_weights((202, 0), n, -8, 0)
    for t in range(3):
        wn = w / w.sum()
        tr.set_weights(wn)
        rec, ferr = tr.round(feature_err=True)
        ferr = ferr.cpu().numpy()
        otr.w = w.copy()
        orec, ost = otr.round()
        assert (np.abs(ferr[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
        assert (np.abs(ferr[:, 1] - ost["err_neg"]) <= err_tolerance(ost["err_neg"], n, "fp32_wide")).all()
        check_stump(rec, ost, orec, otr.vals, labels, wn, n, "fp32_wide")
        w = otr.w.copy()
    tr.close()


def test_strong_classifier_matches_oracle(tiny):
    images, labels, _ = tiny
    say("strong classifier")
    tr = _trainer(images, labels)
    recs = tr.train(5)
    out, score = tr.classify(recs)
    otr = oracle.Trainer(images, labels)
    fv = np.stack([otr.vals[int(r["feature"])] for r in recs])
    ref = oracle.strong_classify(fv, recs["polarity"], recs["threshold"], recs["alpha"])
    assert (out.cpu().numpy() == ref).all()
    tr.close()


def test_wide_keys_fallback_sort():
    # n > 16384 selects 15-bit keys; extreme windows make full-window features
    # span more than 17 bits of value range, forcing the 64-bit sort path
    n = 16500
    rng = np.random.default_rng(7)
    images = np.zeros((n, 24, 24), np.uint8)
    images[: n // 2, :, 12:] = 255          # dark left, bright right
    images[n // 2:, :, :12] = 255           # bright left, dark right
    images[:, 10:12, 10:14] = rng.integers(0, 256, (n, 2, 4))
    labels = (rng.uniform(size=n) < 0.4).astype(np.uint8)
    feats_all = oracle.enumerate_features(24, 24)
    # oracle on a sample of features including the widest ones
    wide = np.nonzero((feats_all[:, 0] == 2) & (feats_all[:, 3] >= 10) & (feats_all[:, 4] >= 20))[0]
    pick = np.unique(np.concatenate([np.arange(0, len(feats_all), 997), [len(feats_all) - 1], wide]))
    say(f"wide keys n={n}: oracle on {len(pick)} features")
    ii = oracle.integrals(images, 0)
    vals = oracle.feature_values(ii, feats_all[pick])
    order = oracle.sort_features(vals)
    assert (vals.max(1) - vals.min(1)).max() >= (1 << 17)
    tr = _trainer(images, labels)
    w = oracle.init_weights(labels)
    wn = w / w.sum()
    rec, ferr = tr.round(feature_err=True)
    ferr = ferr.cpu().numpy()
    ost = oracle.best_stumps(vals, order, labels, wn)
    assert (np.abs(ferr[pick, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
    assert (np.abs(ferr[pick, 1] - ost["err_neg"]) <= err_tolerance(ost["err_neg"], n, "fp32_wide")).all()
    for a in range(0, len(pick), 7):
        j = int(pick[a])
        o, f = tr.sorted(j, 1)
        v = vals[a][o.cpu().numpy()[0]]
        assert (np.diff(v) >= 0).all()
    tr.close()


@pytest.mark.parametrize("W,H", [(13, 19), (24, 10), (5, 32), (32, 7)])
def test_rectangular_windows(W, H):
    """Windows that are not square: integral images, every feature value,
    the sorted keys and two rounds against the oracle."""
    rng = np.random.default_rng(1000 + W * 40 + H)
    n = 700
    images = (rng.integers(0, 6, size=(n, H, W)) * 51).astype(np.uint8)
    labels = (rng.random(n) < 0.4).astype(np.uint8)
    say(f"rectangular windows {W}x{H}")
    otr = oracle.Trainer(images, labels)
    tr = _trainer(images, labels)
    assert tr.F == len(otr.feats) == oracle.feature_count(W, H)
    assert (tr.integral().cpu().numpy() == otr.ii).all()
    assert (tr.feature_values().cpu().numpy() == otr.vals).all()
    order, flags = tr.sorted(0, tr.F)
    v = np.take_along_axis(otr.vals, order.cpu().numpy(), axis=1)
    assert (np.diff(v, axis=1) >= 0).all()
    for t in range(2):
        wn = otr.w / otr.w.sum()
        rec, ferr = tr.round(feature_err=True)
        orec, ost = otr.round()
        ferr = ferr.cpu().numpy()
        assert (np.abs(ferr[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
        assert (np.abs(ferr[:, 1] - ost["err_neg"]) <= err_tolerance(ost["err_neg"], n, "fp32_wide")).all()
        check_stump(rec, ost, orec, otr.vals, labels, wn, n, "fp32_wide")
    tr.close()


@pytest.mark.parametrize("precision", ["fp32_wide", "fp64", "fp32_kahan", "fp32"])
def test_exact_arithmetic_zero_weights_ties(tiny, precision):
    """Dyadic weights with 30 % zeros: prefix sums repeat across many split
    ranks, so every tie-break (smaller error, feature, p = +1, smaller rank)
    decides; with no rounding anywhere both sides must agree bit for bit."""
    images, labels, otr = tiny
    n = len(labels)
    rng = np.random.default_rng(77)
    k = rng.integers(1, 1001, size=n).astype(np.int64)
    k[rng.random(n) < 0.3] = 0
    m = int(np.ceil(np.log2(k.sum())))
    k[int(np.argmax(k))] += (1 << m) - int(k.sum())
    w = k.astype(np.float64) / float(1 << m)
    say(f"exact dyadic weights with zeros, {precision}")
    tr = _trainer(images, labels, precision=precision)
    tr.set_weights(w)
    rec, ferr = tr.round(feature_err=True)
    ferr = ferr.cpu().numpy()
    orec, ost = otr.round(weights=w)
    assert np.array_equal(ferr[:, 0], ost["err_pos"])
    assert np.array_equal(ferr[:, 1], ost["err_neg"])
    assert (rec.feature, rec.polarity, rec.threshold, rec.split_rank) == \
        (orec.feature, orec.polarity, orec.theta, orec.split)
    assert rec.error_raw == orec.err_raw
    assert rec.beta == orec.beta
    assert_weights(tr.weights().cpu().numpy(), otr.w / otr.w.sum(), UPDATE_RTOL, f"zeros {precision}")
    tr.close()


def test_single_positive_window():
    """One positive among many negatives (l = 1): Table 2 gives it weight 1/2."""
    images, labels = synth.small_job((210, 0), 400, 10, 4)
    labels = np.zeros_like(labels)
    labels[123] = 1
    say("one positive window")
    otr = oracle.Trainer(images, labels)
    tr = _trainer(images, labels)
    w = tr.weights().cpu().numpy()
    assert abs(w[123] - 0.5) <= 4e-16 and np.allclose(np.delete(w, 123), 0.5 / 399, rtol=1e-15, atol=0)
    n = len(labels)
    for t in range(3):
        wn = otr.w / otr.w.sum()
        rec, ferr = tr.round(feature_err=True)
        orec, ost = otr.round()
        ferr = ferr.cpu().numpy()
        assert (np.abs(ferr[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
        check_stump(rec, ost, orec, otr.vals, labels, wn, n, "fp32_wide")
    tr.close()


def test_identical_windows_every_feature_constant():
    """Every window the same image: every feature is constant, the only
    splits are k = 0 and k = n, the best error is exactly 1/2 (beta = 1,
    alpha = 0) and the tie-break picks p = +1 at k = 0; weights stay put."""
    # 64 positives and 128 negatives: the Table 2 weights 2^-7 and 2^-8 and
    # the class sums 1/2 are exact in every precision
    n = 192
    images = np.repeat(synth.small_job((220, 0), 1, 12, 8)[0], n, axis=0)
    labels = np.zeros(n, np.uint8)
    labels[np.random.default_rng(220).permutation(n)[:64]] = 1
    tr = _trainer(images, labels)
    w0 = tr.weights().cpu().numpy()
    for t in range(2):
        rec = tr.round()
        assert rec.error_raw == 0.5 and rec.beta == 1.0 and rec.alpha == 0.0
        assert (rec.feature, rec.polarity, rec.split_rank) == (0, 1, 0)
    assert np.allclose(tr.weights().cpu().numpy(), w0, rtol=1e-15, atol=0)
    tr.close()


def test_largest_window_all_types():
    """32 x 32 windows with all five types (the largest feature set)."""
    images, labels = synth.small_job((230, 0), 260, 32, 4)
    say("32x32 windows, all types")
    otr = oracle.Trainer(images, labels)
    tr = _trainer(images, labels)
    assert tr.F == len(otr.feats)
    assert (tr.feature_values().cpu().numpy() == otr.vals).all()
    n = len(labels)
    for t in range(2):
        wn = otr.w / otr.w.sum()
        rec, ferr = tr.round(feature_err=True)
        orec, ost = otr.round()
        ferr = ferr.cpu().numpy()
        assert (np.abs(ferr[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
        assert (np.abs(ferr[:, 1] - ost["err_neg"]) <= err_tolerance(ost["err_neg"], n, "fp32_wide")).all()
        check_stump(rec, ost, orec, otr.vals, labels, wn, n, "fp32_wide")
    tr.close()
