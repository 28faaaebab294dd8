"""The counting sort's tiers at both sides of each boundary (256 x 7, 512 x 7,
1024 x 7, 1024 x 11, 1024 x 15 and 1024 x 31 window slots): each tier skips
the bound check on the slots that every thread fills, so its smallest job is
the case that would expose a slot counted as filled when it is not.  Values,
the full sorted order (ties by internal index: positives first, each class
in caller order) and the run-end flags are compared with the oracle."""
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


@pytest.mark.parametrize("n", [2, 255, 1792, 1793, 3584, 3585, 7168, 7169, 11264, 11265, 15360, 15361])
def test_sort_tier_boundaries(n):
    print(f"sort tier boundary: {n:,} windows of 6x6", flush=True)
    sys.stdout.flush()
    images, labels = synth.small_job((520, n), n, 6, 6)
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels))
    feats = oracle.enumerate_features(6, 6)
    vals = oracle.feature_values(oracle.integrals(images), feats)
    assert tr.F == len(feats)
    assert np.array_equal(tr.feature_values().cpu().numpy(), vals)
    order, flags = tr.sorted(0, tr.F)
    order = order.cpu().numpy().astype(np.int64)
    flags = flags.cpu().numpy().astype(bool)
    # internal index of each caller window: positives first, each class in caller order
    pos = labels == 1
    internal = np.empty(n, np.int64)
    internal[pos] = np.arange(pos.sum())
    internal[~pos] = pos.sum() + np.arange((~pos).sum())
    want = np.lexsort((np.broadcast_to(internal, vals.shape), vals), axis=1)
    assert np.array_equal(order, want)
    v = np.take_along_axis(vals, order, axis=1)
    ends = np.ones_like(flags)
    ends[:, :-1] = np.diff(v, axis=1) != 0
    assert np.array_equal(flags, ends)
    tr.close()
