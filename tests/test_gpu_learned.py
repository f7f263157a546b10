"""Learned tagging end to end on the GPU: training pairs from adaptive runs,
training with the library's kernels, and the gain of the trained network
(committed weights) over criterion tagging every 16 steps, on held-out
seeds."""
import numpy as np
import pytest

from paper_1308_1472_amd import learned as L
from tests.gpu_drive import say

pytestmark = pytest.mark.gpu


def test_collect_pairs_and_short_training():
    say("[learned] collect + train")
    X, Y = L.collect(3, "n+4", nsteps=48, keep_every=1)
    assert X.shape[1] == 16 and len(X) == len(Y) > 100
    assert set(np.unique(Y)) <= {0, 1, 2}
    lev = X[:, 12]
    assert np.all(lev == np.round(lev)) and lev.min() >= L.LMIN and lev.max() <= L.LMAX
    assert np.all(X[:, 13:] == 0)
    net, info = L.train(X, Y, epochs=3, batch=1024)
    assert info["loss_per_epoch"][-1] < 0.8 * info["loss_per_epoch"][0]


def test_learned_tagging_gain():
    """Held-out seeds: learned tags every 16 steps (criterion fallback,
    refinement buffer) stay within 5 % of the criterion every 4 steps in L1
    error against a uniform level-7 run, beat the criterion every 16 steps
    with the same buffer, and regrid 4x less often."""
    net, meta = L.Net.load()
    rows = []
    for s in (180, 181, 182, 183):
        say(f"[learned] compare seed {s}")
        rows.append(L.compare(s, net))
    mean = lambda k: float(np.mean([r[k]["l1_h"] for r in rows]))
    say({k: mean(k) for k in rows[0]})
    assert mean("learned16") <= 1.05 * mean("plain4")
    assert mean("learned16") < mean("plain16")
    for r in rows:
        assert r["learned16"]["regrids"] * 4 <= r["plain4"]["regrids"] + 4
        assert all(v["status"] == 0 for v in r.values())
