"""The strong classifier of Section 2.3 on held-out windows and its error
curve, through the C ABI, against the FP64 oracle's strong classifier run
with the first t stumps for every t."""
import sys

import numpy as np
import pytest

import oracle
from paper_1306_1467_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _job(seed, n_pos, n_neg, flip_seed):
    images, labels = synth.make_job(seed, n_pos, n_neg, size=20, r0=6, contrast=50.0)
    flip = np.random.default_rng(flip_seed).random(len(labels)) < 0.06
    return images, np.where(flip, 1 - labels, labels).astype(np.uint8)


def _oracle_curve(images, labels, recs):
    """Errors of the oracle's strong classifier of the first t stumps, t = 1..T,
    and its decisions with all T."""
    W = images.shape[2]
    feats = np.stack([[r["type"], r["x"], r["y"], r["cell_w"], r["cell_h"]] for r in recs]).astype(np.int32)
    fv = oracle.feature_values(oracle.integrals(images), feats)
    errs = []
    for t in range(1, len(recs) + 1):
        d = oracle.strong_classify(fv[:t], recs["polarity"][:t], recs["threshold"][:t], recs["alpha"][:t])
        errs.append(int(np.sum(d != labels)))
    return np.array(errs, np.int32), d, fv


@pytest.fixture(scope="module")
def trained():
    images, labels = _job((800, 0), 900, 1800, 800)
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision="fp32_kahan")
    recs = tr.train(40)
    yield images, labels, tr, recs
    tr.close()


def test_held_out_curve_matches_oracle(trained):
    _, _, _, recs = trained
    himg, hlab = _job((801, 0), 700, 1300, 801)    # held-out windows of the same recipe
    say(f"held-out: {len(hlab)} windows, {len(recs)} stumps")
    out, score, curve = vb.classify(himg, recs, hlab)
    ref_curve, ref_dec, fv = _oracle_curve(himg, hlab, recs)
    assert np.array_equal(curve.cpu().numpy(), ref_curve)
    assert np.array_equal(out.cpu().numpy(), ref_dec)
    # the score is the alpha of the stumps that vote 1, summed in stump order
    h = recs["polarity"][:, None].astype(np.int64) * fv.astype(np.int64) < \
        (recs["polarity"].astype(np.int64) * recs["threshold"])[:, None]
    s = np.zeros(len(hlab))
    for t in range(len(recs)):
        s = np.where(h[t], s + recs["alpha"][t], s)
    assert np.array_equal(score.cpu().numpy(), s)
    say(f"held-out errors by prefix: first {ref_curve[:3].tolist()}, last {ref_curve[-3:].tolist()}")


def test_training_curve_matches_oracle(trained):
    images, labels, tr, recs = trained
    curve = tr.error_curve(recs).cpu().numpy()
    ref_curve, ref_dec, _ = _oracle_curve(images, labels, recs)
    assert np.array_equal(curve, ref_curve)
    # the context's own classifier agrees with the context-free one on the same windows
    out, _ = tr.classify(recs)
    out2, _, curve2 = vb.classify(images, recs, labels)
    assert np.array_equal(out.cpu().numpy(), ref_dec) and np.array_equal(out2.cpu().numpy(), ref_dec)
    assert np.array_equal(curve2.cpu().numpy(), ref_curve)


@pytest.mark.parametrize("n", [1, 63, 257])
def test_ragged_counts_and_no_labels(trained, n):
    _, _, _, recs = trained
    himg, hlab = _job((802, n), n // 2 + 1, n - n // 2 - 1 if n > 1 else 0, 802)
    himg, hlab = himg[:n], hlab[:n]
    out, score, curve = vb.classify(himg, recs[:7], None)
    assert curve is None
    ref_curve, ref_dec, _ = _oracle_curve(himg, hlab, recs[:7])
    assert np.array_equal(out.cpu().numpy(), ref_dec)
    _, _, curve = vb.classify(himg, recs[:7], hlab)
    assert np.array_equal(curve.cpu().numpy(), ref_curve)


def test_invalid_records_rejected(trained):
    images, labels, _, recs = trained
    bad = recs[:3].copy()
    bad[1]["cell_w"] = 30                        # does not fit a 20x20 window
    with pytest.raises(vb.BoostError) as ei:
        vb.classify(images[:10], bad, labels[:10])
    assert ei.value.code == vb.BOOST_E_INVALID
    bad = recs[:3].copy()
    bad[0]["polarity"] = 0
    with pytest.raises(vb.BoostError):
        vb.classify(images[:10], bad)
    bad = recs[:3].copy()
    bad[2]["alpha"] = np.inf
    with pytest.raises(vb.BoostError):
        vb.classify(images[:10], bad)
    # no stumps: the empty vote is >= half of nothing, every window is 1
    out, score, _ = vb.classify(images[:10], recs[:0])
    assert (out.cpu().numpy() == 1).all() and (score.cpu().numpy() == 0).all()
