"""Measured schedule choice (BOOST_SCHEDULE_AUTO): the tuner times only
schedules that share the job's key layout, its choice changes no result (the
stumps and weights equal those of the chosen schedule run directly, bit for
bit), a job of the same shape takes the cached choice, and a batch tunes each
key format's launch on its own."""
import sys

import numpy as np
import pytest

from paper_1306_1467_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402

# schedule table: (workgroup, units per batch, lanes per feature)
LANES = [16, 16, 16, 16, 16, 32, 64, 16, 16, 16, 16]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(images, labels, rounds, **kw):
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), **kw)
    sched, ms = tr.schedule()
    recs = tr.train(rounds)
    w = tr.weights().cpu().numpy()
    tr.close()
    return sched, ms, recs, w


def test_auto_single_matches_fixed_and_caches():
    vb.boost_tune_cache_clear()
    images, labels = synth.make_job((800, 0), 700, 1300, size=20, r0=6, contrast=70.0)
    say("auto schedule, single job 20x20, 2000 windows")
    sched, ms, recs, w = _run(images, labels, 5, schedule_id=vb.BOOST_SCHEDULE_AUTO)
    assert vb.boost_schedule_count() == len(LANES)
    assert 0 <= sched < len(LANES) and LANES[sched] == 16
    for k, lanes in enumerate(LANES):
        if lanes == 16:
            assert ms[k] > 0, (k, ms)
        else:
            assert ms[k] == -1.0, (k, ms)
    assert ms[sched] == min(m for m in ms if m > 0)
    s2, ms2, recs2, w2 = _run(images, labels, 5, schedule_id=sched)
    assert s2 == sched and all(m == -1.0 for m in ms2)
    assert recs.tobytes() == recs2.tobytes()
    assert np.array_equal(w, w2)
    # same shape again: the cached choice, nothing timed
    s3, ms3, recs3, _ = _run(images, labels, 5, schedule_id=vb.BOOST_SCHEDULE_AUTO)
    assert s3 == sched and all(m == -1.0 for m in ms3)
    assert recs3.tobytes() == recs.tobytes()


def test_auto_batch_per_key_format():
    vb.boost_tune_cache_clear()
    specs = [((810, 0), 6000, 11000, 10, 3, 70.0), ((810, 1), 300, 500, 16, 5, 90.0),
             ((810, 2), 900, 1400, 20, 6, 50.0)]
    data = [synth.make_job(seed, p, m, size=s, r0=r0, contrast=c) for seed, p, m, s, r0, c in specs]
    assert len(data[0][1]) > 16383 >= max(len(d[1]) for d in data[1:])
    say("auto schedule, batch of 3 jobs with both key formats")
    ds = [(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data]
    bt = vb.BatchTrainer(ds, schedule_id=vb.BOOST_SCHEDULE_AUTO)
    (s0, spw0), (s1, spw1) = bt.schedule()
    for s, spw in ((s0, spw0), (s1, spw1)):
        assert 0 <= s < len(LANES) and LANES[s] == 16
        assert spw in (2, 4, 8, 16, 32)
    recs = bt.train(5)
    bt.close()
    # the fixed default schedule gives the same stumps, bit for bit
    bt = vb.BatchTrainer(ds)
    assert bt.schedule() == [(0, 16), (0, 16)]
    ref = bt.train(5)
    bt.close()
    assert recs.tobytes() == ref.tobytes()


def test_batch_schedule_absent_format():
    images, labels = synth.make_job((820, 0), 50, 60, size=12)
    bt = vb.BatchTrainer([(torch.from_numpy(images), torch.from_numpy(labels))])
    assert bt.schedule() == [(0, 16), (-1, 0)]
    with pytest.raises(vb.BoostError):
        vb.boost_batch_get_schedule(bt.ctx, 2)
    bt.close()


def test_stream_probe_changes_nothing():
    images, labels = synth.make_job((830, 0), 500, 900, size=20, r0=6, contrast=40.0)
    ref = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels))
    expect = ref.train(4)
    ref.close()
    for sched in range(vb.boost_schedule_count()):
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), schedule_id=sched)
        first = tr.train(2)
        ms = vb.boost_probe_stream(tr.ctx, 3)
        assert ms > 0
        rest = tr.train(2)
        assert np.concatenate([first, rest]).tobytes() == expect.tobytes(), sched
        tr.close()
    with pytest.raises(vb.BoostError):
        vb.boost_probe_stream(None, 1)
