"""Free-running trajectories against the oracle: both sides train on their own
weights for 50 rounds.  Every round's stump must equal the oracle's, its
error must agree within the tolerance, and the weights must stay normalised,
until a round where the oracle's top two errors tie within the tolerance
(after which two correct trainings may pick different stumps and diverge)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1306_1467_amd import synth
from tests.helpers import assert_weights, err_tolerance, weight_rtol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402

ROUNDS = 50


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp32_wide", "fp64", "fp32_kahan"])
def test_free_running_50_rounds(precision):
    images, labels = synth.make_job((600, 0), 900, 1800, size=20, r0=6, contrast=50.0)
    flip = np.random.default_rng(600).random(len(labels)) < 0.06
    labels = np.where(flip, 1 - labels, labels).astype(np.uint8)
    n = len(labels)
    say(f"{ROUNDS} free-running rounds, {n:,} windows of 20x20, {precision}")
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision)
    recs = tr.train(ROUNDS)
    w_gpu = tr.weights().cpu().numpy()
    tr.close()
    otr = oracle.Trainer(images, labels)
    matched = 0
    betas = []
    for t in range(ROUNDS):
        orec, ost = otr.round()
        g = recs[t]
        assert g["round"] == t
        tol = err_tolerance(np.array([orec.err_raw]), n, precision)[0]
        assert abs(float(g["error_raw"]) - orec.err_raw) <= tol, (t, float(g["error_raw"]), orec.err_raw)
        same = (int(g["feature"]), int(g["polarity"]), int(g["threshold"])) == (orec.feature, orec.polarity, orec.theta)
        if not same:
            errs = np.sort(ost["err"])
            assert errs[1] - errs[0] <= 2 * tol, (t, int(g["feature"]), orec.feature, errs[:2])
            say(f"round {t}: a tie within the tolerance; the trajectories may diverge from here")
            break
        assert abs(float(g["alpha"]) - orec.alpha) <= 1e-6 * abs(orec.alpha) + 1e-12
        betas.append((float(g["beta"]), orec.beta))
        matched += 1
    say(f"{matched} of {ROUNDS} rounds matched the oracle")
    if matched == ROUNDS:
        # the FP64 update, compounded over the rounds: bounded by the betas'
        # differences alone (every other step of the update is FP64 on both sides)
        bg, bo = zip(*betas)
        rtol = weight_rtol(bg, bo)
        say(f"final weights within {rtol:.3g} relative (sum of |ln beta_gpu / beta_oracle|)")
        assert_weights(w_gpu, otr.w / otr.w.sum(), rtol, f"{precision} after {ROUNDS} rounds")
        assert abs(w_gpu.sum() - 1.0) < 1e-12
    assert matched >= 10
