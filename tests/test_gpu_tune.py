"""Tile-shape autotuner: picks a built shape, records it in the cache file, a
new model of the same shape reads it back, and shapes with the same wave
count give bit-identical predictions, including the ping-pong schedule (the
four-wave shape differs only in the order of the output layer's fp32 sum)."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, say, segment_argmin, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,widths", [("bf16", (32, 512, 512, 1)),
                                              ("fp32", (32, 256, 256, 1))])
def test_autotune_picks_and_caches(tmp_path, monkeypatch, precision, widths):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("ADVISOR_TUNE_CACHE", str(cache))
    kd, vd, off = workload.make_descriptors(300, 64, 900, seed=601)
    f, inv = oracle.featurize(kd, vd)
    mu, sd = oracle.zscore_fit(f[inv == 0])
    p = workload.he_init(widths, 602, bias_scale=0.1)
    m = adv.Model(widths, precision)
    m.set_params(p, mu, sd)
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    preds = {}
    for v in (0, 1, 2, 3):
        adv.advisor_model_set_tile_variant(m.handle, v)
        preds[v] = host(m.predict(to_dev(f)))
        b = host(m.rank(K, V, O))
        assert b.tolist() == segment_argmin(np.where(inv == 1, np.nan, preds[v]), off).tolist()
    # same wave count: the same bits whatever the rows per tile or the
    # schedule (shape 3 is the ping-pong schedule of shape 0)
    assert np.array_equal(preds[0].view(np.int32), preds[1].view(np.int32))
    assert np.array_equal(preds[0].view(np.int32), preds[3].view(np.int32))
    assert np.max(np.abs(preds[2] - preds[0]) / np.maximum(np.abs(preds[0]), 1.0)) <= 1e-5
    chosen, times = adv.advisor_autotune(m.handle, K, V, O, reps=3)
    say("autotune %s %s: chose %d, times %s" % (precision, widths, chosen, times[:4]))
    assert chosen in (0, 1, 2, 3) and times[chosen] > 0
    assert times[chosen] == min(t for t in times[:4] if t > 0)
    assert adv.advisor_model_get_tile_variant(m.handle) == chosen
    text = cache.read_text()
    entries = json.loads(text)
    key = [k for k in entries if k.endswith("|%s|%s" % (precision, ",".join(map(str, widths))))]
    assert len(key) == 1 and entries[key[0]] == chosen
    m2 = adv.Model(widths, precision)
    assert adv.advisor_model_get_tile_variant(m2.handle) == chosen


def test_autotune_rejects_unbuilt_shapes(monkeypatch):
    monkeypatch.setenv("ADVISOR_TUNE_CACHE", "")
    m = adv.Model((32, 64, 1), "fp32")
    with pytest.raises(adv.AdvisorError):
        adv.advisor_model_set_tile_variant(m.handle, 1)
    assert adv.advisor_model_get_tile_variant(m.handle) == 0
