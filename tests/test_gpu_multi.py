"""Multi-target ranking (one model per cluster and GPU architecture, as the
paper trains them): every target's row equals a separate advisor_rank with
its model bit for bit, and the fp32 targets' winners match the oracle's."""
import numpy as np
import pytest

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, say, segment_argmin, to_dev

pytestmark = pytest.mark.gpu


def test_rank_multi_equals_separate_calls_and_oracle():
    kd, vd, off = workload.make_descriptors(120, 0, 500, 91, invalid_frac=0.1)
    f, inv = oracle.featurize(kd, vd)
    specs = [((32, 64, 64, 1), "fp32", 92), ((32, 256, 256, 1), "bf16", 93),
             ((32, 48, 24, 40, 1), "fp32", 94)]
    models, params = [], []
    for t, (w, prec, seed) in enumerate(specs):
        p = workload.he_init(w, seed, bias_scale=0.2)
        rows = workload.sample_rows(f.shape[0], 4000, seed)
        ok = f[rows][inv[rows] == 0]
        mu, sd = oracle.zscore_fit(ok)  # each target its own statistics
        m = adv.Model(w, prec)
        m.set_params(p, mu, sd)
        models.append(m)
        params.append((w, p.astype(np.float64), mu, sd))
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    say("rank_multi targets=%d n_v=%d" % (len(models), vd.shape[0]))
    best, pred = adv.advisor_rank_multi([m.handle for m in models], K, V, O, want_pred=True)
    best, pred = host(best), host(pred)
    for t, m in enumerate(models):
        b1, p1 = m.rank(K, V, O, want_pred=True)
        assert np.array_equal(best[t], host(b1))
        assert np.array_equal(pred[t].view(np.uint32), host(p1).view(np.uint32))
        assert np.array_equal(best[t], segment_argmin(pred[t], off))
        w, p64, mu, sd = params[t]
        if specs[t][1] == "fp32":
            rb, rp = oracle.rank(kd, vd, off, w, p64, mu, sd)
            agree = np.mean(best[t] == rb)
            say("  target %d: fp32 argmin agreement with the oracle %.4f" % (t, agree))
            assert agree >= 0.99


def test_rank_multi_grouped_pass_equals_separate_calls():
    """Targets whose models share precision, tile width and Z-score
    statistics (the statistics describe the variants, not the machine) run
    in grouped passes that build each input tile once: nine paper-sized
    targets sharing statistics (two groups, eight and one), one with its own
    statistics, one of another precision and two bf16x3 targets (a group of
    their own). Every row equals a separate
    advisor_rank bit for bit, predictions included."""
    kd, vd, off = workload.make_descriptors(400, 0, 700, 95, invalid_frac=0.05)
    f, inv = oracle.featurize(kd, vd)
    ok = f[inv == 0]
    mu, sd = oracle.zscore_fit(ok[:20000])
    mu2, sd2 = oracle.zscore_fit(ok[20000:40000])
    specs = [((32, 64, 128, 64, 32, 1), "fp32", 100 + t, mu, sd) for t in range(9)]
    specs += [((32, 64, 128, 64, 32, 1), "fp32", 120, mu2, sd2),
              ((32, 64, 128, 64, 32, 1), "bf16", 121, mu, sd),
              ((32, 48, 24, 40, 1), "fp32", 122, mu, sd),   # same tile width 64
              ((32, 64, 128, 64, 32, 1), "bf16x3", 123, mu, sd),   # a bf16x3 group of two
              ((32, 64, 128, 64, 32, 1), "bf16x3", 124, mu, sd)]
    models = []
    for w, prec, seed, m_, s_ in specs:
        m = adv.Model(w, prec)
        m.set_params(workload.he_init(w, seed, bias_scale=0.2), m_, s_)
        models.append(m)
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    best, pred = adv.advisor_rank_multi([m.handle for m in models], K, V, O, want_pred=True)
    best, pred = host(best), host(pred)
    for t, m in enumerate(models):
        b1, p1 = m.rank(K, V, O, want_pred=True)
        assert np.array_equal(best[t], host(b1)), t
        assert np.array_equal(pred[t].view(np.uint32), host(p1).view(np.uint32)), t
    # the grouped rows are not copies of one another
    assert not np.array_equal(pred[0], pred[1])
    # the fp32 paper-sized targets agree with the oracle
    for t in (0, 8, 9):
        w, _, seed, m_, s_ = specs[t]
        rb, _ = oracle.rank(kd, vd, off, w, workload.he_init(w, seed, bias_scale=0.2)
                            .astype(np.float64), m_, s_)
        agree = float(np.mean(best[t] == rb))
        say("grouped target %d: argmin agreement with the oracle %.4f" % (t, agree))
        assert agree >= 0.99
    for m in models:
        m.close()
