"""Batched jobs: every job's stumps and weights equal those of the same job
trained alone through the single-job path (bit for bit), for uneven sizes,
window sizes and key formats; and the batched stumps are valid against the
oracle on small jobs."""
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


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _plain(images, labels, rounds, **kw):
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), **kw)
    recs = tr.train(rounds)
    w = tr.weights().cpu().numpy()
    tr.close()
    return recs, w


def _datasets(specs):
    return [synth.make_job(seed, p, m, size=s, r0=r0, contrast=c) for seed, p, m, s, r0, c in specs]


@pytest.mark.parametrize("precision", ["fp32_wide", "fp32_kahan", "fp64", "fp32"])
def test_batch_equals_plain_uneven(precision):
    specs = [((700, 0), 300, 600, 24, 7, 80.0), ((700, 1), 40, 90, 16, 5, 120.0),
             ((700, 2), 1500, 3000, 20, 6, 60.0), ((700, 3), 5, 7, 12, 4, 90.0),
             ((700, 4), 800, 1200, 28, 9, 140.0)]
    data = _datasets(specs)
    say(f"batch of {len(data)} uneven jobs, {precision}")
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data], precision=precision)
    rounds = 6
    brecs = bt.train(rounds)
    assert brecs.shape == (rounds, len(data))
    for k, (images, labels) in enumerate(data):
        precs, pw = _plain(images, labels, rounds, precision=precision)
        assert brecs[:, k].tobytes() == precs.tobytes(), k
        assert np.array_equal(bt.weights(k).cpu().numpy(), pw), k
    bt.close()


def test_batch_mixed_key_formats():
    # one job above 16,383 windows uses 15-bit keys; the batch mixes formats
    specs = [((710, 0), 6000, 11000, 10, 3, 70.0), ((710, 1), 100, 150, 12, 4, 90.0),
             ((710, 2), 900, 700, 10, 3, 50.0)]
    data = _datasets(specs)
    assert len(data[0][1]) > 16383
    say("batch with mixed key formats")
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data])
    brecs = bt.train(4)
    for k, (images, labels) in enumerate(data):
        precs, pw = _plain(images, labels, 4)
        assert brecs[:, k].tobytes() == precs.tobytes(), k
        assert np.array_equal(bt.weights(k).cpu().numpy(), pw), k
    bt.close()


@pytest.mark.parametrize("precision,sched", [("fp32_wide", 9), ("fp32_kahan", 9), ("fp32_wide", 10)])
def test_batch_rotating_loads(precision, sched):
    # schedules 9 and 10 (rotating loads) in the batched kernel, both key
    # formats, against each job alone under the default schedule
    specs = [((720, 0), 300, 600, 24, 7, 80.0), ((720, 1), 3, 4, 8, 2, 90.0),
             ((720, 2), 6000, 11000, 10, 3, 70.0), ((720, 3), 700, 500, 16, 5, 60.0)]
    data = _datasets(specs)
    say(f"batch with rotating loads, {precision}, schedule {sched}")
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data], precision=precision,
                         schedule_id=sched)
    assert [s for s, _ in bt.schedule()] == [sched, sched]
    brecs = bt.train(4)
    for k, (images, labels) in enumerate(data):
        precs, pw = _plain(images, labels, 4, precision=precision)
        assert brecs[:, k].tobytes() == precs.tobytes(), k
        assert np.array_equal(bt.weights(k).cpu().numpy(), pw), k
    bt.close()


def test_batch_graph_direct_timing_agree():
    data = _datasets([((720, 0), 200, 300, 16, 5, 40.0), ((720, 1), 350, 250, 20, 6, 35.0)])
    say("batch: graph vs direct vs timing")
    out = []
    for flags in (0, vb.BOOST_FLAG_NO_GRAPH, vb.BOOST_FLAG_TIMING):
        bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data], flags=flags)
        out.append(bt.train(7))
        if flags == vb.BOOST_FLAG_TIMING:
            t = bt.timing()
            assert t[2] == 7 and t[0] > 0
        bt.close()
    assert out[0].tobytes() == out[1].tobytes() == out[2].tobytes()


def test_batch_stumps_valid_against_oracle():
    data = _datasets([((730, 0), 60, 70, 12, 4, 30.0), ((730, 1), 33, 41, 8, 2, 60.0)])
    say("batch vs oracle")
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data])
    brecs = bt.train(3)
    for k, (images, labels) in enumerate(data):
        otr = oracle.Trainer(images, labels)
        n = len(labels)
        for t in range(3):
            wn = otr.w / otr.w.sum()
            orec, ost = otr.round()
            g = brecs[t, k]
            tol = err_tolerance(np.array([orec.err_raw]), n, "fp32_wide")[0]
            assert abs(float(g["error_raw"]) - orec.err_raw) <= tol
            e = stump_error(otr.vals[int(g["feature"])], labels, wn, int(g["polarity"]), int(g["threshold"]))
            assert abs(e - orec.err_raw) <= tol
    bt.close()


def test_batch_rejects_bad_jobs():
    images, labels = synth.make_job((740,), 10, 10, size=8)
    with pytest.raises(vb.BoostError):
        vb.BatchTrainer([(torch.from_numpy(images), torch.from_numpy(np.ones_like(labels)))])
    with pytest.raises(vb.BoostError):
        vb.BatchTrainer([(torch.from_numpy(images[:1]), torch.from_numpy(labels[:1]))])
