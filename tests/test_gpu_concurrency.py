"""Independent contexts: jobs trained on their own streams, interleaved from
one thread or driven from several host threads at once, give exactly the
records and weights of the same jobs trained alone.  (A context must not be
used from two threads at once; different contexts may be.)"""
import sys
import threading

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


def _jobs():
    specs = [((900, 0), 400, 700, 20, 6, 45.0, "fp32_wide"), ((900, 1), 1200, 900, 16, 5, 35.0, "fp32_kahan"),
             ((900, 2), 300, 500, 24, 7, 60.0, "fp64"), ((900, 3), 6000, 11000, 12, 4, 50.0, "fp32_wide")]
    return [(synth.make_job(seed, p, m, size=s, r0=r0, contrast=c), prec) for seed, p, m, s, r0, c, prec in specs]


def _alone(data, rounds):
    out = []
    for (images, labels), prec in data:
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=prec)
        out.append((tr.train(rounds), tr.weights().cpu().numpy()))
        tr.close()
    return out


def test_interleaved_streams_match_alone():
    data = _jobs()
    rounds = 6
    ref = _alone(data, rounds)
    say("interleaved rounds of 4 contexts on 4 streams")
    trs = [vb.Trainer(torch.from_numpy(i), torch.from_numpy(l), precision=p) for (i, l), p in data]
    recs = [[] for _ in trs]
    for t in range(rounds):
        for k, tr in enumerate(trs):
            recs[k].append(tr.round())
    for k, tr in enumerate(trs):
        got = np.array([(r.feature, r.polarity, r.threshold, r.split_rank) for r in recs[k]])
        exp = np.stack([ref[k][0]["feature"], ref[k][0]["polarity"], ref[k][0]["threshold"], ref[k][0]["split_rank"]], 1)
        assert np.array_equal(got, exp), k
        assert np.array_equal([r.error_raw for r in recs[k]], ref[k][0]["error_raw"]), k
        assert np.array_equal(tr.weights().cpu().numpy(), ref[k][1]), k
        tr.close()


def test_host_threads_match_alone():
    data = _jobs()
    rounds = 8
    ref = _alone(data, rounds)
    say("4 host threads, one context each, trained at once")
    results = [None] * len(data)
    errors = []

    def work(k):
        try:
            (images, labels), prec = data[k]
            tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=prec,
                            schedule_id=vb.BOOST_SCHEDULE_AUTO)
            results[k] = (tr.train(rounds), tr.weights().cpu().numpy())
            tr.close()
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((k, repr(e)))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(data))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=240)
    assert not errors, errors
    for k in range(len(data)):
        assert results[k] is not None, k
        assert results[k][0].tobytes() == ref[k][0].tobytes(), k
        assert np.array_equal(results[k][1], ref[k][1]), k
