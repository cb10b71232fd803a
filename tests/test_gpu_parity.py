"""GPU parity of the HIP path against the float64 CPU oracle.

Integer stages (features, invalid flags, argmin indices) must match bit for
bit; fp32 predictions within 1e-5 relative (|p - r| / max(|r|, 1) on the
predicted ln-runtime); bf16 predictions are checked against a bound derived
from bf16 rounding and their argmin agreement is reported. Shapes span
several tiles with ragged tails, empty segments and invalid variants.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import dev, host, rel_err, say, segment_argmin, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _desc(nk, lo, hi, seed, depth=3, invalid_frac=0.0, empty=()):
    kd, vd, off = workload.make_descriptors(nk, lo, hi, seed, depth=depth,
                                            invalid_frac=invalid_frac)
    if empty:
        counts = off[1:] - off[:-1]
        keep = np.ones(vd.shape[0], dtype=bool)
        for k in empty:
            keep[off[k]:off[k + 1]] = False
            counts[k] = 0
        vd = vd[keep]
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return kd, vd, off


def _model(widths, precision, seed, kd, vd, bias=0.2):
    p = workload.he_init(widths, seed, bias_scale=bias)
    f, inv = oracle.featurize(kd, vd)
    mu, sd = oracle.zscore_fit(f[inv == 0])
    m = adv.Model(widths, precision)
    m.set_params(p, mu, sd)
    return m, p.astype(np.float64), mu, sd


@pytest.mark.parametrize("depth,invalid", [(3, 0.0), ("mixed", 0.2), (4, 0.05), (1, 0.1)])
def test_featurize_bit_exact(depth, invalid):
    kd, vd, off = _desc(300, 1, 700, seed=101, depth=depth, invalid_frac=invalid)
    say("featurize depth=%s invalid=%s n_v=%d" % (depth, invalid, vd.shape[0]))
    f_ref, inv_ref = oracle.featurize(kd, vd)
    f, inv = adv.advisor_featurize(to_dev(kd), to_dev(vd))
    assert np.array_equal(host(f), f_ref)
    assert np.array_equal(host(inv), inv_ref)


def test_featurize_wraparound_and_edges():
    # values beyond 2^63 wrap identically; one-row and 257-row (ragged) inputs
    kd = np.array([[4, 4096, 4096, 4096, 4096, 4, 64, 1, 1, 1, 1, 1024, 3, 3, 3, 3],
                   [2, 7, 9, 1, 1, 0, 3, 0, 0, 0, 0, 0, 0, 0, 0, 0]], dtype=np.int64)
    vd = np.array([[0, 4, 1, 1, 3, 3, 3, 3], [1, 2, 3, 5, 0, 0, 0, 0], [1, 3, 3, 5, 0, 0, 0, 0]],
                  dtype=np.int64)
    f_ref, inv_ref = oracle.featurize(kd, vd)
    f, inv = adv.advisor_featurize(to_dev(kd), to_dev(vd))
    assert np.array_equal(host(f), f_ref) and np.array_equal(host(inv), inv_ref)
    kd, vd, off = _desc(3, 257, 257, seed=5)
    vd = vd[:257]
    f_ref, inv_ref = oracle.featurize(kd, vd)
    f, inv = adv.advisor_featurize(to_dev(kd), to_dev(vd))
    assert np.array_equal(host(f), f_ref) and np.array_equal(host(inv), inv_ref)


def test_zscore_fit_matches_oracle():
    kd, vd, off = _desc(200, 16, 600, seed=7)
    f_ref, inv = oracle.featurize(kd, vd)
    mu_ref, sd_ref = oracle.zscore_fit(f_ref)
    mu, sd = adv.advisor_zscore_fit(to_dev(f_ref))
    assert np.allclose(host(mu), mu_ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(host(sd), sd_ref, rtol=1e-12, atol=1e-12)
    # constant columns are detected exactly
    assert np.array_equal(host(sd) == 1.0, sd_ref == 1.0)


def _brute(pred, off):
    out = []
    for k in range(off.size - 1):
        seg = [(pred[i], i) for i in range(off[k], off[k + 1]) if not np.isnan(pred[i])]
        out.append(min(seg)[1] if seg else -1)
    return out


def test_rank_preds_bit_exact_edge_patterns():
    rng = np.random.default_rng(3)
    vals = np.array([np.nan, -1.5, -0.0, 0.0, 2.0, np.inf, -np.inf], dtype=np.float32)
    n = 5000
    pred = vals[rng.integers(0, vals.size, n)]
    cuts = np.sort(rng.integers(0, n + 1, size=900))
    off = np.concatenate([[0], cuts, [n]]).astype(np.int64)   # many empty segments
    best = host(adv.advisor_rank_preds(to_dev(pred), to_dev(off)))
    assert best.tolist() == oracle.argmin(pred.astype(np.float64), off).tolist()
    # signed zero: -0 and +0 tie, lowest index wins
    pz = np.array([0.0, -0.0, 1.0, -0.0, 0.0], dtype=np.float32)
    best = host(adv.advisor_rank_preds(to_dev(pz), to_dev(np.array([0, 2, 5]))))
    assert best.tolist() == [0, 3]


def test_rank_preds_long_segments():
    rng = np.random.default_rng(4)
    pred = rng.standard_normal(200000).astype(np.float32)
    pred[rng.random(pred.size) < 0.01] = np.nan
    off = np.array([0, 3, 100000, 100001, 200000], dtype=np.int64)
    best = host(adv.advisor_rank_preds(to_dev(pred), to_dev(off)))
    assert best.tolist() == oracle.argmin(pred.astype(np.float64), off).tolist()


def test_rank_preds_chunked_long_segments():
    """Kernels of 16384 or more variants on average take the chunked form
    (waves over fixed chunks of variants, per-kernel atomic minima of the
    keys): segment ends on and off the chunk boundaries, empty and all-NaN
    segments, short segments among long ones, and equal values spread over
    many chunks (the lowest index must still win), against the oracle."""
    rng = np.random.default_rng(6)
    n = 1_500_000
    pred = np.round(rng.standard_normal(n), 1).astype(np.float32)  # many ties
    pred[rng.random(n) < 0.01] = np.nan
    cuts = [0, 5, 5, 16384, 16385, 32768, 200000, 200000, 200003, 700000, 1_000_000]
    pred[200000:200003] = np.nan                       # an all-NaN segment
    pred[900000] = -7.0                                # one clear winner
    pred[[400000, 650000]] = -9.0                      # a tie across chunks
    pred[-1] = -0.0
    off = np.array(cuts + [n], dtype=np.int64)
    assert n >= 16384 * (off.size - 1)
    say("argmin chunked: %d kernels, %d variants" % (off.size - 1, n))
    best = host(adv.advisor_rank_preds(to_dev(pred), to_dev(off)))
    assert best.tolist() == oracle.argmin(pred.astype(np.float64), off).tolist()
    assert best[1] == -1 and best[6] == -1 and best[7] == -1  # empty, empty, all NaN
    assert best[8] == 400000 and best[9] == 900000


@pytest.mark.parametrize("widths", [(32, 64, 64, 1), (32, 256, 256, 256, 1), (32, 8, 1),
                                    (32, 48, 24, 40, 1), (32, 512, 512, 1),
                                    (32, 1024, 1024, 1)])
def test_predict_fp32_within_tolerance(widths):
    kd, vd, off = _desc(40, 16, 300, seed=11)
    m, p, mu, sd = _model(widths, "fp32", 21, kd, vd)
    f_ref, inv = oracle.featurize(kd, vd)
    f_ref = f_ref[inv == 0]
    say("predict fp32 widths=%s n=%d" % (widths, f_ref.shape[0]))
    pred = host(m.predict(to_dev(f_ref)))
    ref = oracle.forward(widths, p, oracle.normalize(f_ref, mu, sd))
    err = rel_err(pred, ref)
    say("  max rel err %.3g" % err.max())
    assert err.max() <= FP32_TOL


@pytest.mark.parametrize("precision,widths", [("fp32", (32, 256, 256, 256, 1)),
                                              ("fp32", (32, 64, 64, 1)),
                                              ("bf16", (32, 512, 512, 512, 512, 1)),
                                              ("bf16", (32, 64, 64, 1))])
def test_rank_against_oracle(precision, widths):
    kd, vd, off = _desc(120, 1, 900, seed=31, invalid_frac=0.05, empty=(3, 50, 119))
    vd[5, 0] = (vd[5, 0] + 1) % 120          # a variant filed under the wrong kernel
    m, p, mu, sd = _model(widths, precision, 41, kd, vd)
    say("rank %s widths=%s n_v=%d" % (precision, widths, vd.shape[0]))
    best_ref, pred_ref = oracle.rank(kd, vd, off, widths, p, mu, sd)
    best, pred = m.rank(to_dev(kd), to_dev(vd), to_dev(off), want_pred=True)
    best, pred = host(best), host(pred)
    # ineligible variants (invalid or in the wrong segment) are NaN on both sides
    assert np.array_equal(np.isnan(pred), np.isnan(pred_ref))
    ok = ~np.isnan(pred_ref)
    err = rel_err(pred[ok], pred_ref[ok])
    # the GPU's argmin is exact on its own predictions
    assert best.tolist() == segment_argmin(pred, off).tolist()
    agree = np.mean(best == best_ref)
    say("  max rel err %.3g  argmin agreement %.4f" % (err.max(), agree))
    if precision == "fp32":
        assert err.max() <= FP32_TOL
    else:
        # bf16 rounding of inputs, weights and activations: about 2^-8 relative
        # per layer, a few percent at the output for these random networks
        assert err.max() <= 0.1
    assert best[3] == -1 and best[50] == -1 and best[119] == -1
    # the standalone prediction entry point gives the same bits
    f, inv = oracle.featurize(kd, vd)
    pred2 = host(m.predict(to_dev(f)))
    assert np.array_equal(pred2[ok], pred[ok])


def test_rank_deterministic_and_permutation_invariant():
    widths = (32, 256, 256, 256, 1)
    kd, vd, off = _desc(64, 16, 400, seed=51)
    m, p, mu, sd = _model(widths, "fp32", 52, kd, vd)
    b1, p1 = m.rank(to_dev(kd), to_dev(vd), to_dev(off), want_pred=True)
    b2, p2 = m.rank(to_dev(kd), to_dev(vd), to_dev(off), want_pred=True)
    assert torch.equal(b1, b2) and torch.equal(p1.view(torch.int32), p2.view(torch.int32))
    # permuting rows inside segments permutes predictions bit for bit, even
    # though the rows land in other tiles
    rng = np.random.default_rng(2)
    perm = np.concatenate([off[k] + rng.permutation(off[k + 1] - off[k]) for k in range(64)])
    b3, p3 = m.rank(to_dev(kd), to_dev(vd[perm]), to_dev(off), want_pred=True)
    assert np.array_equal(host(p3).view(np.int32), host(p1)[perm].view(np.int32))


def test_rank_empty_and_tiny():
    widths = (32, 64, 64, 1)
    kd, vd, off = _desc(4, 1, 3, seed=61)
    m, p, mu, sd = _model(widths, "fp32", 62, kd, vd)
    # no variants at all: every kernel gets -1
    best = m.rank(to_dev(kd), to_dev(vd[:0]), to_dev(np.zeros(5, dtype=np.int64)))
    assert host(best).tolist() == [-1, -1, -1, -1]
    best_ref, _ = oracle.rank(kd, vd, off, widths, p, mu, sd)
    best = m.rank(to_dev(kd), to_dev(vd), to_dev(off))
    assert host(best).tolist() == best_ref.tolist()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_rank_segments_spanning_many_tiles(precision):
    """Kernels whose variants span thousands of tiles (and tiles holding the
    ends of several kernels): the fused argmin, folded per tile and run and
    merged by atomics across workgroups, must equal the exact segment argmin
    of the same call's own predictions, with the winner inside its segment."""
    widths = (32, 64, 64, 1)
    rng = np.random.default_rng(91)
    counts = np.array([700000, 1, 0, 3, 300001, 129, 0, 64], dtype=np.int64)
    nk = counts.size
    kd, vd, _ = workload.make_descriptors(nk, 16, 17, 92)
    # variant rows drawn from a small pool, so exact ties recur across tiles
    pool = np.concatenate([vd[vd[:, 0] == k][:8] for k in range(nk)])
    rows = []
    for k, c in enumerate(counts):
        mine = pool[pool[:, 0] == k]
        rows.append(mine[rng.integers(0, mine.shape[0], c)])
    V = np.concatenate(rows)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    m, p, mu, sd = _model(widths, precision, 93, kd, V)
    pred = torch.empty(V.shape[0], dtype=torch.float32, device="cuda")
    best_t, _ = m.rank(to_dev(kd), to_dev(V), to_dev(off), pred_out=pred)
    best = host(best_t)
    ref = segment_argmin(host(pred), off)
    say("%s rank over segments of up to %d variants: %s" % (precision, counts.max(), best.tolist()))
    assert best.tolist() == ref.tolist()
    for k in range(nk):
        if best[k] >= 0:
            assert off[k] <= best[k] < off[k + 1]
        else:
            assert counts[k] == 0 or np.isnan(host(pred)[off[k]:off[k + 1]]).all()


def test_validate_offsets_and_debug_mode(monkeypatch):
    """The segmentation check names the lowest offending entry; with
    ADVISOR_DEBUG_OFFSETS set the ranking calls fail on malformed offsets
    instead of ranking them."""
    good = np.array([0, 3, 3, 10], dtype=np.int64)
    assert adv.advisor_validate_offsets(to_dev(good), 10) == -1
    assert adv.advisor_validate_offsets(to_dev(good), 11) == 3          # last != n_v
    assert adv.advisor_validate_offsets(to_dev(np.array([1, 3, 3, 10])), 10) == 0
    assert adv.advisor_validate_offsets(to_dev(np.array([0, 5, 3, 10])), 10) == 1
    assert adv.advisor_validate_offsets(to_dev(np.zeros(1, dtype=np.int64)), 0) == -1
    big = np.arange(0, 200001, dtype=np.int64)
    big[150000] = big[149999] - 1                                       # dips below its left neighbour
    assert adv.advisor_validate_offsets(to_dev(big), 200000) == 149999
    widths = (32, 64, 64, 1)
    kd, vd, off = _desc(3, 4, 9, seed=95)
    m, p, mu, sd = _model(widths, "fp32", 96, kd, vd)
    bad_off = off.copy()
    bad_off[1], bad_off[2] = bad_off[2], bad_off[1]
    if bad_off[1] == bad_off[2]:
        bad_off[1] += 1
    monkeypatch.setenv("ADVISOR_DEBUG_OFFSETS", "1")
    m.rank(to_dev(kd), to_dev(vd), to_dev(off))                         # valid: ranks
    with pytest.raises(adv.AdvisorError):
        m.rank(to_dev(kd), to_dev(vd), to_dev(bad_off))
    with pytest.raises(adv.AdvisorError):
        adv.advisor_rank_preds(torch.zeros(vd.shape[0], device="cuda"), to_dev(bad_off))
    monkeypatch.setenv("ADVISOR_DEBUG_OFFSETS", "0")
    m.rank(to_dev(kd), to_dev(vd), to_dev(bad_off))                     # unchecked: clamps, no error
    m.close()
