"""Incremental retraining (boost_extend): a context extended by new windows
equals a fresh boost_init on the concatenated windows, bit for bit -- integral
images, every feature value, the sorted keys and run ends of every feature,
the initial weights, and a 5-round trajectory (records and weights).  Unions
of 7,169 to 15,360 windows that add at most 256 are merged from the old
keys; the others are sorted in full, and both are checked."""
import sys

import numpy as np
import pytest

from paper_1306_1467_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _data(seed, n_pos, n_neg, size, shuffle=True):
    images, labels = synth.make_job(seed, n_pos, n_neg, size=size, r0=max(2, size // 4), contrast=50.0)
    flip = np.random.default_rng(seed[0] + 7).random(len(labels)) < 0.05
    labels = np.where(flip, 1 - labels, labels).astype(np.uint8)
    if shuffle:
        p = np.random.default_rng(seed[0] + 9).permutation(len(labels))
        images, labels = images[p], labels[p]
    return np.ascontiguousarray(images), np.ascontiguousarray(labels)


def _tr(images, labels, **kw):
    return vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), **kw)


def _same(ext, fresh, all_values=True):
    assert ext.n == fresh.n and ext.F == fresh.F
    assert np.array_equal(ext.integral().cpu().numpy(), fresh.integral().cpu().numpy())
    if all_values:
        assert np.array_equal(ext.feature_values().cpu().numpy(), fresh.feature_values().cpu().numpy())
    step = 20000
    for j0 in range(0, ext.F, step):
        nf = min(step, ext.F - j0)
        oe, fe = ext.sorted(j0, nf)
        of, ff = fresh.sorted(j0, nf)
        assert np.array_equal(oe.cpu().numpy(), of.cpu().numpy()), j0
        assert np.array_equal(fe.cpu().numpy(), ff.cpu().numpy()), j0
    assert np.array_equal(ext.weights().cpu().numpy(), fresh.weights().cpu().numpy())
    ra, rb = ext.train(5), fresh.train(5)
    assert ra.tobytes() == rb.tobytes()
    assert np.array_equal(ext.weights().cpu().numpy(), fresh.weights().cpu().numpy())


@pytest.mark.parametrize("n0,m", [(8000, 80), (8000, 256), (8000, 257), (8000, 800), (8000, 4000), (2000, 20)])
@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32_wide"])
def test_extend_equals_fresh(n0, m, precision):
    old_img, old_lab = _data((950,), 7 * n0 // 20, n0 - 7 * n0 // 20, 12)
    new_img, new_lab = _data((951,), m // 3 + 1, m - m // 3 - 1, 12)
    say(f"extend 12x12: {n0} + {m} windows, {precision}")
    base = _tr(old_img, old_lab, precision=precision)
    base.train(3)                      # a base that has trained: extension starts over on the union
    ext = base.extend(new_img, new_lab)
    assert ext.merged() == (n0 + m > 7168 and m <= 256)   # the others are sorted in full
    fresh = _tr(np.concatenate([old_img, new_img]), np.concatenate([old_lab, new_lab]), precision=precision)
    _same(ext, fresh)
    for t in (base, ext, fresh):
        t.close()


@pytest.mark.parametrize("case", ["one_window", "all_new_positive", "all_new_negative", "auto_schedule"])
def test_extend_edge_cases(case):
    old_img, old_lab = _data((952,), 2800, 4600, 12)
    if case == "one_window":
        new_img, new_lab = _data((953,), 1, 0, 12)
    elif case == "all_new_positive":
        new_img, new_lab = _data((954,), 150, 0, 12, shuffle=False)
        new_lab[:] = 1
    elif case == "all_new_negative":
        new_img, new_lab = _data((955,), 0, 150, 12, shuffle=False)
        new_lab[:] = 0
    else:
        new_img, new_lab = _data((956,), 50, 150, 12)
    kw = {"schedule_id": vb.BOOST_SCHEDULE_AUTO} if case == "auto_schedule" else {}
    say(f"extend edge case {case}: 7400 + {len(new_lab)}")
    base = _tr(old_img, old_lab, **kw)
    ext = base.extend(new_img, new_lab)
    assert ext.merged()
    fresh = _tr(np.concatenate([old_img, new_img]), np.concatenate([old_lab, new_lab]), **kw)
    _same(ext, fresh)
    for t in (base, ext, fresh):
        t.close()


def test_extend_headline_size_and_the_full_sort_beyond_the_merge_range():
    """24x24 windows at the benchmark's scale: 14,800 + 200 (merged, 15 window
    slots a thread), 10,000 + 5,000 (sorted in full: more than 256 new), and
    15,000 + 500 (beyond 15,360 windows: sorted in full); sorted keys and
    trajectories equal a fresh init."""
    images, labels = synth.workload_jobs("faces15k")[0].make()
    p = np.random.default_rng(957).permutation(len(labels))
    images, labels = np.ascontiguousarray(images[p]), np.ascontiguousarray(labels[p])
    extra_img, extra_lab = _data((958,), 200, 300, 24)
    for n0, new_img, new_lab, merged in ((14800, images[14800:], labels[14800:], True),
                                        (10000, images[10000:], labels[10000:], False),
                                        (15000, extra_img, extra_lab, False)):
        old_img, old_lab = (images[:n0], labels[:n0]) if n0 < 15000 else (images, labels)
        say(f"extend 24x24: {n0} + {len(new_lab)}")
        base = _tr(np.ascontiguousarray(old_img), np.ascontiguousarray(old_lab), precision="fp32_kahan")
        ext = base.extend(np.ascontiguousarray(new_img), np.ascontiguousarray(new_lab))
        assert ext.merged() == merged
        fresh = _tr(np.concatenate([old_img, new_img]), np.concatenate([old_lab, new_lab]), precision="fp32_kahan")
        _same(ext, fresh, all_values=False)
        vals_e = ext.feature_values(0, 4096).cpu().numpy()
        assert np.array_equal(vals_e, fresh.feature_values(0, 4096).cpu().numpy())
        for t in (base, ext, fresh):
            t.close()
        del base, ext, fresh
        torch.cuda.empty_cache()


def test_extend_rejects_bad_arguments():
    old_img, old_lab = _data((959,), 20, 30, 8)
    base = _tr(old_img, old_lab)
    bad = np.array([0, 2, 1], np.uint8)
    with pytest.raises(vb.BoostError) as ei:
        base.extend(old_img[:3], bad)
    assert ei.value.code == vb.BOOST_E_INVALID
    with pytest.raises(ValueError):
        base.extend(np.zeros((2, 9, 8), np.uint8), np.zeros(2, np.uint8))
    assert vb.boost_extend_workspace_bytes(base.ctx, 0) == 0
    assert vb.boost_extend_workspace_bytes(base.ctx, 32767) == 0
    base.close()
