"""Parity at the full workload sizes, in the launch configurations the
benchmark times: every tile shape built for the width, and the captured plan.
The oracle recomputes a seeded sample of whole kernels one by one; properties
that hold at any size (exact argmin on the library's own predictions, every
winner inside its segment, replay bits equal to eager bits, gradient
additivity over a batch split) are checked on the whole output.

Workloads: 4096 kernels x U[16,1024] variants through 32-256x3-1 in fp32;
16384 kernels x U[64,1024] through 32-512x4-1 in bf16; 32768 kernels x
U[128,1024] through 32-1024x4-1 in fp8; a training step on a batch of 65,536
rows of 32-512x4-1 in bf16."""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, rel_err, say, segment_argmin, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _statistics(kd, vd, seed):
    """Z-score statistics from the oracle's features of a seeded row sample."""
    rows = workload.sample_rows(vd.shape[0], 65536, seed)
    f, inv = oracle.featurize(kd, vd[rows])
    return oracle.zscore_fit(f[inv == 0])


def _oracle_sample(kd, vd, off, widths, p64, mu, sd, n_kernels, seed):
    """The oracle's ranking of a seeded sample of whole kernels, mapped back
    to global variant indices."""
    ks, rows, sub_off = workload.sample_kernels(off, n_kernels, seed)
    vsub = vd[rows].copy()
    vsub[:, 0] = np.repeat(np.arange(ks.size), np.diff(sub_off))
    best, pred = oracle.rank(kd[ks], vsub, sub_off, widths, p64, mu, sd)
    glob = np.where(best >= 0, rows[np.maximum(best, 0)], -1)
    return ks, rows, glob, pred


def _check_whole_output(best, pred, off):
    """Exact argmin of the library's own predictions, each winner inside its
    segment, on every kernel."""
    assert np.array_equal(best, segment_argmin(pred, off))
    k = np.nonzero(best >= 0)[0]
    assert np.all(best[k] >= off[k]) and np.all(best[k] < off[k + 1])


def _run_config(cfg, precision, n_sample, pred_check, monkeypatch):
    monkeypatch.setenv("ADVISOR_TUNE_CACHE", "")  # no tuning file written
    c = workload.make_config(cfg)
    kd, vd, off, widths = c["kdesc"], c["vdesc"], c["offsets"], c["widths"]
    p = c["params"]
    mu, sd = _statistics(kd, vd, 7000 + cfg)
    m = adv.Model(widths, precision)
    m.set_params(p, mu, sd)
    if precision == "fp8":
        rows = workload.sample_rows(vd.shape[0], 65536, 7100 + cfg)
        f, inv = oracle.featurize(kd, vd[rows])
        m.calibrate_fp8(to_dev(f[inv == 0]))
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    ks, rows, best_ref, pred_ref = _oracle_sample(kd, vd, off, widths, p.astype(np.float64), mu,
                                                  sd, n_sample, 7200 + cfg)
    say("cfg%d %s: %d kernels, %d variants; oracle sample %d kernels, %d variants" %
        (cfg, precision, kd.shape[0], vd.shape[0], ks.size, rows.size))
    ok = ~np.isnan(pred_ref)
    results = {}
    for shape in (0, 1, 2, 3):
        try:
            adv.advisor_model_set_tile_variant(m.handle, shape)
        except adv.AdvisorError:
            continue
        best, pred = m.rank(K, V, O, want_pred=True)
        best, pred = host(best), host(pred)
        _check_whole_output(best, pred, off)
        ps = pred[rows]
        assert np.array_equal(np.isnan(ps), ~ok)
        err = rel_err(ps[ok], pred_ref[ok])
        agree = float(np.mean(best[ks] == best_ref))
        say("  tile shape %d: max rel err %.3g, median %.3g, argmin agreement %.4f" %
            (shape, err.max(), np.median(err), agree))
        pred_check(err, agree)
        results[shape] = (best, pred)
    assert results
    # the tile shapes give each row the same hidden activations. Shapes with
    # the same waves per tile also share the output layer's summation order:
    # 0, 1 and 3 (the ping-pong schedule of shape 0) for fp32 and bf16; 1 and
    # 3 for fp8, whose shape 0 has four waves. The same bits; otherwise only
    # that fp32 summation order differs.
    same = {0, 1, 3} if precision != "fp8" else {1, 3}
    ref = min(s for s in results if s in same) if same & set(results) else None
    for s, (b, pr) in results.items():
        if s in same and s != ref:
            assert np.array_equal(b, results[ref][0])
            assert np.array_equal(pr.view(np.int32), results[ref][1].view(np.int32))
        elif s != ref:
            base = results[ref if ref is not None else min(results)][1]
            assert np.nanmax(rel_err(pr, base)) <= 1e-5
    # the captured plan of the tuned shape replays the eager bits
    chosen, _ = adv.advisor_autotune(m.handle, K, V, O, reps=2)
    best_buf = torch.empty(kd.shape[0], dtype=torch.int64, device="cuda")
    pred_buf = torch.empty(vd.shape[0], dtype=torch.float32, device="cuda")
    plan = adv.Plan.rank(m, K, V, O, best_buf, pred_buf)
    for _ in range(2):
        plan.launch()
        assert np.array_equal(host(best_buf), results[chosen][0])
        assert np.array_equal(host(pred_buf).view(np.int32), results[chosen][1].view(np.int32))
    plan.close()
    m.close()


def test_rank_fullsize_fp32_batched(monkeypatch):
    def check(err, agree):
        assert err.max() <= FP32_TOL
        # a flip needs two variants within 2e-5 of each other on ln(us)
        assert agree >= 0.99
    _run_config(2, "fp32", 64, check, monkeypatch)


def test_rank_fullsize_bf16(monkeypatch):
    def check(err, agree):
        # bf16 rounding of inputs, weights and activations (8-bit mantissas)
        assert err.max() <= 0.1 and np.median(err) <= 0.01
        assert agree >= 0.8
    _run_config(3, "bf16", 32, check, monkeypatch)


def test_rank_fullsize_fp8(monkeypatch):
    def check(err, agree):
        # e4m3 operands (3-bit mantissas) in the three square layers
        assert np.median(err) <= 0.05
        assert agree >= 0.5
    _run_config(5, "fp8", 16, check, monkeypatch)


def test_train_step_fullsize_bf16():
    """One step at batch 65,536: sampled predictions against the oracle, and
    the gradient of the whole batch equal to the mean of the gradients of its
    two halves (the step's reductions are exact sums up to fp32 rounding)."""
    c = workload.make_config(4)
    kd, vd, widths, p = c["kdesc"], c["vdesc"], c["widths"], c["params"]
    f, inv = oracle.featurize(kd, vd)
    f = f[inv == 0]
    rows = workload.sample_rows(f.shape[0], 65536, 7400)
    f = f[rows]
    mu, sd = oracle.zscore_fit(f)
    y = 10.0 + 3.0 * workload.noise(f.shape[0], 7401)
    F, Y = to_dev(f), to_dev(y)
    n = f.shape[0]
    assert n == 65536

    def grads(a, b):
        m = adv.Model(widths, "bf16")
        m.set_params(p, mu, sd)
        # a fresh model per call: the gradient is taken at the initial weights
        loss, gn = adv.advisor_train_step(m.handle, F[a:b].contiguous(), Y[a:b].contiguous())
        g = torch.empty(m.param_count, dtype=torch.float32, device="cuda")
        adv.advisor_model_grads(m.handle, g)
        out = host(loss)[0], host(gn)[0], host(g).astype(np.float64)
        m.close()
        return out

    loss, gn, g = grads(0, n)
    l1, _, g1 = grads(0, n // 2)
    l2, _, g2 = grads(n // 2, n)
    say("train fullsize: loss %.6f halves %.6f %.6f  gnorm %.6f" % (loss, l1, l2, gn))
    assert abs(loss - 0.5 * (l1 + l2)) <= 1e-9 * loss
    assert abs(gn - np.linalg.norm(g)) <= 1e-9 * gn
    assert np.linalg.norm(g - 0.5 * (g1 + g2)) <= 1e-4 * np.linalg.norm(g)
    # sampled rows of the forward pass against the oracle
    m = adv.Model(widths, "bf16")
    m.set_params(p, mu, sd)
    yhat, _ = adv.advisor_mlp_forward(m.handle, F)
    s = workload.sample_rows(n, 512, 7402)
    ref = oracle.forward(widths, p.astype(np.float64), oracle.normalize(f[s], mu, sd))
    err = rel_err(host(yhat)[s], ref)
    say("  forward sample: max rel err %.3g median %.3g" % (err.max(), np.median(err)))
    assert err.max() <= 0.1 and np.median(err) <= 0.01
