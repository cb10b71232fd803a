"""bf16x3 models on the GPU against the float64 oracle.

A bf16x3 model keeps every weight and activation as a pair of bf16 values
(the bf16 rounding hi of the fp32 value and the rounding lo of the
remainder) and forms each product as hi*hi + hi*lo + lo*hi on the bf16
matrix cores, accumulating in fp32. Each operand's pair is within 2^-18 of
it (relative) and the dropped lo*lo is below 2^-18 of the product, so a
product carries at most about 3 * 2^-18 (1.1e-5) relative error where fp32
carries 2^-24: close to the fp32 path at bf16 speed. The tests bound the
prediction error on ln(us) against the oracle, require the argmin to be
exact on the library's own predictions, and require it to match the oracle
wherever the oracle's best two variants are further apart than that error
can bridge."""
import numpy as np
import pytest

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, rel_err, say, segment_argmin, to_dev

pytestmark = pytest.mark.gpu

# about three times the largest errors measured on these networks (maximum
# 7.4e-5, medians 4e-6 to 6e-6 on ln(us)); fp32's own bound is 1e-5
X3_MAX = 2.5e-4
X3_MEDIAN = 2e-5


def _model(widths, seed, kd, vd):
    p = workload.he_init(widths, seed, bias_scale=0.2)
    f, inv = oracle.featurize(kd, vd)
    mu, sd = oracle.zscore_fit(f[inv == 0])
    m = adv.Model(widths, "bf16x3")
    m.set_params(p, mu, sd)
    return m, p.astype(np.float64), mu, sd


def _margin(pred, off):
    """Per kernel: gap between its best and second-best eligible prediction
    (inf with fewer than two)."""
    out = np.full(off.size - 1, np.inf)
    for k in range(off.size - 1):
        v = pred[off[k]:off[k + 1]]
        v = np.sort(v[~np.isnan(v)])
        if v.size >= 2:
            out[k] = v[1] - v[0]
    return out


@pytest.mark.parametrize("widths", [(32, 64, 128, 64, 32, 1), (32, 256, 256, 256, 1),
                                    (32, 512, 512, 512, 512, 1), (32, 64, 64, 1)])
def test_bf16x3_rank_against_oracle(widths):
    # three kernels without variants, 5% invalid variants
    counts = np.random.default_rng(30).integers(1, 901, size=120)
    counts[[3, 50, 119]] = 0
    kd, vd, off = workload.make_descriptors(120, 1, 900, 31, depth=3, invalid_frac=0.05,
                                            counts=counts)
    vd[5, 0] = (vd[5, 0] + 1) % 120          # a variant filed under the wrong kernel
    m, p, mu, sd = _model(widths, 41, kd, vd)
    best_ref, pred_ref = oracle.rank(kd, vd, off, widths, p, mu, sd)
    best, pred = m.rank(to_dev(kd), to_dev(vd), to_dev(off), want_pred=True)
    best, pred = host(best), host(pred)
    assert np.array_equal(np.isnan(pred), np.isnan(pred_ref))
    ok = ~np.isnan(pred_ref)
    err = rel_err(pred[ok], pred_ref[ok])
    assert best.tolist() == segment_argmin(pred, off).tolist()
    empty = np.diff(off) == 0
    assert np.all(best[empty] == -1) and np.array_equal(best[empty], best_ref[empty])
    gap = _margin(pred_ref, off) / np.maximum(np.abs(np.nan_to_num(
        pred_ref[np.maximum(best_ref, 0)])), 1.0)
    clear = gap > 2 * X3_MAX
    agree = float(np.mean(best == best_ref))
    say("bf16x3 widths=%s n_v=%d: max rel err %.3g, median %.3g, argmin agreement %.4f "
        "(%d of %d kernels clear of near-ties)" % (widths, vd.shape[0], err.max(), np.median(err),
                                                   agree, int(clear.sum()), clear.size))
    assert err.max() <= X3_MAX and np.median(err) <= X3_MEDIAN
    assert np.array_equal(best[clear], best_ref[clear])
    # the feature-input entry point gives the same bits
    f, _ = oracle.featurize(kd, vd)
    assert np.array_equal(host(m.predict(to_dev(f)))[ok], pred[ok])
    m.close()


def test_bf16x3_full_width_against_oracle():
    """The 32-1024x4-1 network on a ragged batch spanning many tiles."""
    widths = (32, 1024, 1024, 1024, 1024, 1)
    kd, vd, off = workload.make_descriptors(24, 1, 600, 77, depth="mixed")
    m, p, mu, sd = _model(widths, 78, kd, vd)
    best_ref, pred_ref = oracle.rank(kd, vd, off, widths, p, mu, sd)
    best, pred = m.rank(to_dev(kd), to_dev(vd), to_dev(off), want_pred=True)
    best, pred = host(best), host(pred)
    ok = ~np.isnan(pred_ref)
    assert np.array_equal(np.isnan(pred), ~ok)
    err = rel_err(pred[ok], pred_ref[ok])
    say("bf16x3 1024-wide n_v=%d: max rel err %.3g, median %.3g, argmin agreement %.4f"
        % (vd.shape[0], err.max(), np.median(err), float(np.mean(best == best_ref))))
    assert err.max() <= X3_MAX and np.median(err) <= X3_MEDIAN
    assert best.tolist() == segment_argmin(pred, off).tolist()
    m.close()


def test_bf16x3_refuses_training():
    m = adv.Model((32, 64, 1), "bf16x3")
    x = to_dev(np.zeros((16, 32), dtype=np.int64))
    y = to_dev(np.zeros(16, dtype=np.float64))
    with pytest.raises(adv.AdvisorError):
        adv.advisor_train_step(m.handle, x, y)
    m.close()
