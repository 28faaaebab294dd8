"""Size limits: the largest job (32,767 windows, which fills the 15-bit key
format and its 32,768-entry weight table), the boundary between the 14-bit
and 15-bit key formats (16,383 / 16,384 windows), the largest job the
counting sort takes with 31 windows a thread (31,744) and the first one past
it (31,745), a job in between (24,000), and the FP64 table limit (20,000
windows).  Values, sorted keys and two teacher-forced rounds are
compared with the oracle (FP32 weights with FP64 or compensated sums; plain
FP32 is covered at small sizes, where its error bound is tight)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1306_1467_amd import synth
from tests.helpers import check_stump, err_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1467_amd import vjboost as vb  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[32767, 31745, 31744, 24000, 16384, 16383])
def big(request):
    n = request.param
    images, labels = synth.small_job((500, n), n, 6, 8)
    say(f"oracle for {n:,} windows of 6x6")
    return images, labels, oracle.Trainer(images, labels)


@pytest.mark.parametrize("precision", ["fp32_wide", "fp32_kahan"])
def test_limits(big, precision):
    images, labels, otr = big
    n = len(labels)
    say(f"{n:,} windows, {precision}")
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision)
    assert tr.F == len(otr.feats)
    assert (tr.feature_values().cpu().numpy() == otr.vals).all()
    order, flags = tr.sorted(0, tr.F)
    order = order.cpu().numpy()
    flags = flags.cpu().numpy().astype(bool)
    assert (np.sort(order, axis=1) == np.arange(n)[None, :]).all()
    v = np.take_along_axis(otr.vals, order, axis=1)
    d = np.diff(v, axis=1)
    assert (d >= 0).all()
    ends = np.ones_like(flags)
    ends[:, :-1] = d != 0
    assert (flags == ends).all()
    w = oracle.init_weights(labels)
    for t in range(2):
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


def test_fp64_table_limit():
    images, labels = synth.small_job((510, 0), 20001, 4, 8)
    with pytest.raises(vb.BoostError):
        vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision="fp64")
    images, labels = images[:20000], labels[:20000]
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision="fp64")
    otr = oracle.Trainer(images, labels)
    wn = otr.w / otr.w.sum()
    rec, ferr = tr.round(feature_err=True)
    orec, ost = otr.round()
    n = len(labels)
    assert (np.abs(ferr.cpu().numpy()[:, 0] - ost["err_pos"]) <= err_tolerance(ost["err_pos"], n, "fp64")).all()
    check_stump(rec, ost, orec, otr.vals, labels, wn, n, "fp64")
    tr.close()
