"""Batched workloads at full size, in the configuration the benchmark times
(measured schedule choice, graph replay): the 32 uneven jobs of 24x24
windows, and the largest 15-bit-key job of the 64-job mixed workload with
smaller jobs of every window size.  Sampled jobs are compared with the same
job run alone (bit for bit) and, on sampled features, with the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1306_1467_amd import synth
from tests.helpers import err_tolerance, stump_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402

ROUNDS = 4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check_jobs(specs, data, check_idx):
    say(f"batch of {len(data)} jobs, {sum(s.n for s in specs):,} windows in all")
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data],
                         schedule_id=vb.BOOST_SCHEDULE_AUTO)
    recs = bt.train(ROUNDS)
    weights = {k: bt.weights(k).cpu().numpy() for k in check_idx}
    bt.close()
    del bt
    torch.cuda.empty_cache()
    for k in check_idx:
        images, labels = data[k]
        n = len(labels)
        say(f"job {k}: {specs[k].size}x{specs[k].size}, {n:,} windows, alone")
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), schedule_id=vb.BOOST_SCHEDULE_AUTO)
        alone = tr.train(ROUNDS)
        w_alone = tr.weights().cpu().numpy()
        assert recs[:, k].tobytes() == alone.tobytes(), k
        assert np.array_equal(weights[k], w_alone), k
        # the oracle on sampled features, teacher-forced with the oracle's own weights
        feats = oracle.enumerate_features(specs[k].size, specs[k].size)
        rng = np.random.default_rng(40 + k)
        pick = np.sort(rng.choice(len(feats), 600, replace=False))
        ii = oracle.integrals(images)
        w = oracle.init_weights(labels)
        for t in range(2):
            wn = w / w.sum()
            tr.set_weights(wn)
            rec, ferr = tr.round(feature_err=True)
            ferr = ferr.cpu().numpy()
            sel = np.unique(np.concatenate([pick, [rec.feature]]))
            vals = oracle.feature_values(ii, feats[sel])
            ost = oracle.best_stumps(vals, oracle.sort_features(vals), labels, wn)
            assert (np.abs(ferr[sel, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp32_wide")).all()
            assert (np.abs(ferr[sel, 1] - ost["err_neg"]) <= err_tolerance(ost["err_neg"], n, "fp32_wide")).all()
            a = int(np.nonzero(sel == rec.feature)[0][0])
            e = stump_error(vals[a], labels, wn, rec.polarity, rec.threshold)
            assert abs(e - rec.error_raw) <= err_tolerance(np.array([e]), n, "fp32_wide")[0]
            assert rec.error_raw <= ost["err"].min() + err_tolerance(np.array([ost["err"].min()]), n, "fp32_wide")[0]
            # the oracle's update of these weights by the GPU's stump, for the next round
            h = (rec.polarity * vals[a].astype(np.int64) < rec.polarity * rec.threshold).astype(np.int64)
            eps = max(e, 1e-10)
            w = wn * np.where(h == labels.astype(np.int64), eps / (1 - eps), 1.0)
        tr.close()
        del tr
        torch.cuda.empty_cache()


def test_batch32_fullsize():
    specs = synth.workload_jobs("batch32")
    data = [s.make() for s in specs]
    order = np.argsort([s.n for s in specs])
    _check_jobs(specs, data, [int(order[0]), int(order[-1])])


def test_batch64_largest_wide_job_with_every_window_size():
    specs = synth.workload_jobs("batch64")
    wide = [k for k, s in enumerate(specs) if s.n > 16383]
    big = max(wide, key=lambda k: specs[k].n)
    pick = [big]
    for size in (16, 20, 24, 28):
        pick.append(min((k for k, s in enumerate(specs) if s.size == size and k != big), key=lambda k: specs[k].n))
    sub = [specs[k] for k in pick]
    data = [s.make() for s in sub]
    _check_jobs(sub, data, [0, 4])


@pytest.mark.parametrize("precision", ["fp32_kahan"])
def test_batch64_every_job_equals_plain(precision):
    """All 64 jobs of the mixed-window batched workload (windows 16 to 28,
    1,000 to 8,000 positives and 2,000 to 20,000 negatives per job, 14- and
    15-bit keys), in its own precision mode and the measured schedule choice:
    every job's records and weights after 4 batched rounds equal those of the
    job trained alone, bit for bit."""
    specs = synth.workload_jobs("batch64")
    say(f"batch64: generating {len(specs)} jobs")
    data = [s.make() for s in specs]
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data], precision=precision,
                         schedule_id=vb.BOOST_SCHEDULE_AUTO)
    say(f"batch64 {precision}: schedules {bt.schedule()}")
    recs = bt.train(ROUNDS)
    weights = [bt.weights(k).cpu().numpy() for k in range(len(data))]
    bt.close()
    del bt
    torch.cuda.empty_cache()
    for k, (images, labels) in enumerate(data):
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision,
                        schedule_id=vb.BOOST_SCHEDULE_AUTO)
        alone = tr.train(ROUNDS)
        w_alone = tr.weights().cpu().numpy()
        tr.close()
        del tr
        assert recs[:, k].tobytes() == alone.tobytes(), k
        assert np.array_equal(weights[k], w_alone), k
        if k % 16 == 15:
            say(f"jobs 0..{k} equal alone")
            torch.cuda.empty_cache()
