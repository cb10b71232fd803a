"""Precision-refined ranking: a bf16 or fp8 first pass over every variant,
then each kernel's top-k candidates re-ranked by an fp32 model of the same
weights. Checked exactly against its definition (numpy over the library's
own predictions: the top-k set by the first pass, the winner by the second),
and against the fp32 ranking and the float64 oracle for agreement."""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, say, segment_argmin, to_dev

pytestmark = pytest.mark.gpu


def _expected(pred_lo, pred_hi, off, k):
    """Per kernel: the k smallest (pred_lo, index) among non-NaN rows, then
    the smallest (pred_hi, index) among those; -1 if none."""
    out = np.full(off.size - 1, -1, dtype=np.int64)
    for s in range(off.size - 1):
        idx = np.arange(off[s], off[s + 1])
        idx = idx[~np.isnan(pred_lo[idx])]
        if idx.size == 0:
            continue
        order = np.lexsort((idx, pred_lo[idx].astype(np.float64)))
        cand = idx[order[:k]]
        cand = cand[~np.isnan(pred_hi[cand])]
        if cand.size == 0:
            continue
        o2 = np.lexsort((cand, pred_hi[cand].astype(np.float64)))
        out[s] = cand[o2[0]]
    return out


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_refined_rank_definition_and_agreement(precision):
    widths = (32, 256, 256, 256, 1)
    kd, vd, off = workload.make_descriptors(300, 1, 900, seed=701, invalid_frac=0.05)
    counts = np.diff(off)
    keep = np.ones(vd.shape[0], dtype=bool)
    for k in (7, 150):                      # two empty kernels
        keep[off[k]:off[k + 1]] = False
        counts[k] = 0
    vd = vd[keep]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    vd[3, 0] = (vd[3, 0] + 1) % 300         # a variant filed under the wrong kernel
    f, inv = oracle.featurize(kd, vd)
    mu, sd = oracle.zscore_fit(f[inv == 0])
    p = workload.he_init(widths, 702, bias_scale=0.2)
    lo = adv.Model(widths, precision)
    lo.set_params(p, mu, sd)
    if precision == "fp8":
        lo.calibrate_fp8(to_dev(f[inv == 0][:4096]))
    hi = adv.Model(widths, "fp32")
    hi.set_params(p, mu, sd)
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    best_hi, pred_hi = hi.rank(K, V, O, want_pred=True)
    best_hi, pred_hi = host(best_hi), host(pred_hi)
    best_ref, _ = oracle.rank(kd, vd, off, widths, p.astype(np.float64), mu, sd)
    pred_lo = torch.empty(vd.shape[0], dtype=torch.float32, device="cuda")
    for k in (1, 2, 4, 8, 16):
        best = host(lo.rank_refined(hi, K, V, O, top_k=k, pred_out=pred_lo))
        pl = host(pred_lo)
        assert np.array_equal(best, _expected(pl, pred_hi, off, k))
        if k == 1:
            assert np.array_equal(best, segment_argmin(pl, off))
        assert best[7] == -1 and best[150] == -1
        a_hi = float(np.mean(best == best_hi))
        a_ref = float(np.mean(best == best_ref))
        say("%s refined top_k=%d: agreement with fp32 rank %.4f, with the oracle %.4f" %
            (precision, k, a_hi, a_ref))
    # the fp32 winner is essentially always among the bf16 top 8 (measured
    # 1.0 here); fp8's 3-bit mantissas scatter the predictions more, so it
    # needs 16 candidates for the same (measured 0.993 at 8, 1.0 at 16)
    k_needed = 8 if precision == "bf16" else 16
    bestk = host(lo.rank_refined(hi, K, V, O, top_k=k_needed))
    assert np.mean(bestk == best_hi) >= 0.995


def test_refined_rank_argument_checks():
    m = adv.Model((32, 64, 1), "bf16")
    h = adv.Model((32, 64, 1), "fp32")
    kd = torch.zeros((1, 16), dtype=torch.int64, device="cuda")
    vd = torch.zeros((4, 8), dtype=torch.int64, device="cuda")
    off = torch.tensor([0, 4], dtype=torch.int64, device="cuda")
    for bad_k in (0, 3, 32):
        with pytest.raises(adv.AdvisorError):
            adv.advisor_rank_refined(m.handle, h.handle, kd, vd, off, top_k=bad_k)
    # all four variants invalid (kernel row of zeros): no winner
    best = adv.advisor_rank_refined(m.handle, h.handle, kd, vd, off, top_k=4)
    assert host(best).tolist() == [-1]
