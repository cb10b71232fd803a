"""GPU training path against the float64 oracle: gradients of the hand-written
backward, the float64 loss and gradient norm, the Adam update, determinism,
checkpoint/resume, the torch.autograd.Function wrapper, and what training
gains over an untrained network or an unranked variant list."""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import elementwise_grad_err as _elementwise, host, say, to_dev
from oracle import cost

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    kd, vd, off = workload.make_descriptors(max(8, n // 300), 16, 1024, seed)
    f, inv = oracle.featurize(kd, vd)
    f = f[inv == 0]
    rows = workload.sample_rows(f.shape[0], n, seed + 1)
    f = f[rows]
    mu, sd = oracle.zscore_fit(f)
    y = cost.target(f, workload.noise(f.shape[0], seed + 2))
    return f, y, mu, sd


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))




@pytest.mark.parametrize("widths", [(32, 64, 64, 1), (32, 256, 256, 256, 1), (32, 48, 24, 40, 1),
                                    (32, 8, 1), (32, 512, 512, 1), (32, 1024, 1)])
def test_backward_fp32_matches_oracle(widths):
    f, y, mu, sd = _batch(1500, 301)
    p = workload.he_init(widths, 302, bias_scale=0.1)
    m = adv.Model(widths, "fp32")
    m.set_params(p, mu, sd)
    yhat, saved = adv.advisor_mlp_forward(m.handle, to_dev(f))
    n = f.shape[0]
    dy = (2.0 * (yhat.double() - to_dev(y)) / n).float()
    g = host(adv.advisor_mlp_backward(m.handle, dy, saved, n))
    x = oracle.normalize(f, mu, sd)
    loss_ref, g_ref = oracle.loss_grad(widths, p.astype(np.float64), x, y)
    err = _rel(g, g_ref)
    ew = _elementwise(g, g_ref, widths)
    say("backward fp32 %s: rel grad err %.2e, worst element %.2e" % (widths, err, ew))
    assert err <= 1e-4
    # element by element: fp32 sums of 1500 rows of products that carry the
    # forward's and backward's own fp32 rounding (relative ~1e-6 per value)
    assert ew <= 2e-3
    # every layer on its own, not only the whole vector
    off = 0
    for i in range(len(widths) - 1):
        k = widths[i + 1] * widths[i] + widths[i + 1]
        assert _rel(g[off:off + k], g_ref[off:off + k]) <= 1e-3
        off += k


@pytest.mark.parametrize("widths", [(32, 64, 64, 1), (32, 256, 256, 1), (32, 1024, 1024, 1)])
def test_backward_bf16_close_to_oracle(widths):
    """bf16 activations and weights (8-bit mantissas) through forward and
    backward, a ragged batch (1500 rows, padded to 1536 inside), every tile
    width class of the backward kernel (64: fewer transposed units than
    threads; 1024: 64-row tiles)."""
    f, y, mu, sd = _batch(1500, 341)
    p = workload.he_init(widths, 342, bias_scale=0.1)
    m = adv.Model(widths, "bf16")
    m.set_params(p, mu, sd)
    yhat, saved = adv.advisor_mlp_forward(m.handle, to_dev(f))
    n = f.shape[0]
    dy = (2.0 * (yhat.double() - to_dev(y)) / n).float()
    g = host(adv.advisor_mlp_backward(m.handle, dy, saved, n))
    x = oracle.normalize(f, mu, sd)
    loss_ref, g_ref = oracle.loss_grad(widths, p.astype(np.float64), x, y)
    err = _rel(g, g_ref)
    ew = _elementwise(g, g_ref, widths)
    say("backward bf16 %s: rel grad err %.2e, worst element %.2e" % (widths, err, ew))
    assert np.isfinite(g).all()
    # a few bf16 roundings (unit roundoff 2^-9) per product; measured ~2e-3
    assert err <= 1e-2
    # element by element, each operand of every product rounded to 8
    # significant bits (relative 2^-9 = 2e-3 per rounding, a few per path)
    assert ew <= 0.1


def _one_step(precision, widths, n, seed):
    f, y, mu, sd = _batch(n, seed)
    p = workload.he_init(widths, seed + 10, bias_scale=0.1)
    m = adv.Model(widths, precision)
    m.set_params(p, mu, sd)
    loss, gnorm = adv.advisor_train_step(m.handle, to_dev(f), to_dev(y), lr=1e-3)
    g = torch.empty(m.param_count, dtype=torch.float32, device="cuda")
    adv.advisor_model_grads(m.handle, g)
    w_new, _, _ = m.get_params()
    x = oracle.normalize(f, mu, sd)
    loss_ref, g_ref = oracle.loss_grad(widths, p.astype(np.float64), x, y)
    return m, p, host(loss)[0], host(gnorm)[0], host(g), w_new, loss_ref, g_ref


def test_train_step_fp32_matches_oracle():
    widths = (32, 256, 256, 256, 1)
    m, p, loss, gnorm, g, w_new, loss_ref, g_ref = _one_step("fp32", widths, 3000, 311)
    say("fp32 step: loss %.6f ref %.6f  gnorm %.6f ref %.6f" % (loss, loss_ref, gnorm,
                                                              oracle.l2norm(g_ref)))
    assert abs(loss - loss_ref) / loss_ref <= 1e-5
    assert _rel(g, g_ref) <= 1e-4
    ew = _elementwise(g, g_ref, widths)
    say("fp32 step: worst gradient element %.2e" % ew)
    assert ew <= 2e-3
    # the float64 norm is the norm of the gradient the step used
    assert abs(gnorm - np.linalg.norm(g.astype(np.float64))) <= 1e-12 * gnorm
    assert abs(gnorm - oracle.l2norm(g_ref)) / oracle.l2norm(g_ref) <= 1e-4
    # Adam on the gradient the GPU used, in float64, from m = v = 0 at t = 1
    w = p.astype(np.float64)
    mm = np.zeros_like(w)
    vv = np.zeros_like(w)
    oracle.adam(w, mm, vv, g.astype(np.float64), 1, lr=1e-3)
    step = w_new.astype(np.float64) - p
    assert np.max(np.abs(step - (w - p))) <= 1e-3 * 1e-3   # |step| <= lr; error far below it
    big = np.abs(g) > 1e-4 * np.abs(g).max()
    assert np.allclose(step[big], (w - p)[big], rtol=1e-3, atol=1e-7)


def test_train_step_bf16_close_to_oracle():
    widths = (32, 512, 512, 512, 512, 1)
    m, p, loss, gnorm, g, w_new, loss_ref, g_ref = _one_step("bf16", widths, 2048, 321)
    err = _rel(g, g_ref)
    say("bf16 step: loss %.5f ref %.5f  rel grad err %.3e" % (loss, loss_ref, err))
    assert abs(loss - loss_ref) / loss_ref <= 2e-2
    assert err <= 5e-2
    ew = _elementwise(g, g_ref, widths)
    say("bf16 step: worst gradient element %.2e" % ew)
    assert ew <= 0.25
    assert np.isfinite(w_new).all()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_steps_deterministic_and_resumable(precision):
    widths = (32, 128, 128, 1)
    f, y, mu, sd = _batch(4000, 331)
    p = workload.he_init(widths, 332)
    F, Y = to_dev(f), to_dev(y)
    a = adv.Model(widths, precision)
    a.set_params(p, mu, sd)
    for _ in range(3):
        adv.advisor_train_step(a.handle, F, Y)
    b = adv.Model(widths, precision)
    b.set_params(p, mu, sd)
    for _ in range(3):
        adv.advisor_train_step(b.handle, F, Y)
    wa, _, _ = a.get_params()
    wb, _, _ = b.get_params()
    assert np.array_equal(wa.view(np.int32), wb.view(np.int32))
    # checkpoint after 2 steps, resume in a fresh model, 1 more step
    c = adv.Model(widths, precision)
    c.set_params(p, mu, sd)
    for _ in range(2):
        adv.advisor_train_step(c.handle, F, Y)
    wc, muc, sdc = c.get_params()
    am, av, t = adv.advisor_model_get_adam(c.handle)
    assert t == 2
    d = adv.Model(widths, precision)
    d.set_params(wc, muc, sdc)
    adv.advisor_model_set_adam(d.handle, am, av, t)
    adv.advisor_train_step(d.handle, F, Y)
    wd, _, _ = d.get_params()
    assert np.array_equal(wa.view(np.int32), wd.view(np.int32))


def test_autograd_function_matches_oracle():
    widths = (32, 64, 64, 1)
    f, y, mu, sd = _batch(1200, 341)
    p = workload.he_init(widths, 342, bias_scale=0.1)
    m = adv.Model(widths, "fp32")
    m.set_params(p, mu, sd)
    params = torch.tensor(p, device="cuda", requires_grad=True)
    yhat = adv.mlp(params, to_dev(f), m)
    loss = ((yhat.double() - to_dev(y)) ** 2).mean()
    loss.backward()
    x = oracle.normalize(f, mu, sd)
    loss_ref, g_ref = oracle.loss_grad(widths, p.astype(np.float64), x, y)
    assert abs(loss.item() - loss_ref) / loss_ref <= 1e-5
    assert _rel(host(params.grad), g_ref) <= 1e-4
    assert _elementwise(host(params.grad), g_ref, widths) <= 2e-3
    # torch's own Adam drives the library's forward and backward
    opt = torch.optim.Adam([params], lr=1e-3)
    first = None
    for _ in range(30):
        opt.zero_grad()
        lo = ((adv.mlp(params, to_dev(f), m).double() - to_dev(y)) ** 2).mean()
        first = lo.item() if first is None else first
        lo.backward()
        opt.step()
    assert lo.item() < first


def _regret_stats(t, off, pick):
    return cost.regret(t, off, pick)


def test_training_gains_over_untrained_and_unranked():
    """Train on synthetic runtimes of 1024 kernels, rank 256 held-out kernels:
    the trained network's picks have lower true-runtime regret than the first
    listed variant, a random variant, and the untrained network's pick."""
    widths = (32, 256, 256, 256, 1)
    kd, vd, off = workload.make_descriptors(1024, 64, 512, 351)
    f, inv = oracle.featurize(kd, vd)
    f = f[inv == 0]
    mu, sd = oracle.zscore_fit(f)
    y = cost.target(f, workload.noise(f.shape[0], 352))
    p0 = workload.he_init(widths, 353)
    m = adv.Model(widths, "bf16")
    m.set_params(p0, mu, sd)
    untrained = adv.Model(widths, "bf16")
    untrained.set_params(p0, mu, sd)
    F, Y = to_dev(f), to_dev(y)
    rng = np.random.default_rng(354)
    B = 8192
    first_loss = None
    for it in range(600):
        idx = torch.from_numpy(rng.integers(0, f.shape[0], B)).cuda()
        loss, _ = adv.advisor_train_step(m.handle, F[idx].contiguous(), Y[idx].contiguous(), lr=2e-3)
        if first_loss is None:
            first_loss = host(loss)[0]
    last_loss = host(loss)[0]
    say("gain test: loss %.3f -> %.4f" % (first_loss, last_loss))
    # held-out kernels
    kh, vh, oh = workload.make_descriptors(256, 64, 512, 355)
    fh, invh = oracle.featurize(kh, vh)
    assert not invh.any()
    t = cost.runtime_s(fh)
    best = host(m.rank(to_dev(kh), to_dev(vh), to_dev(oh)))
    best_u = host(untrained.rank(to_dev(kh), to_dev(vh), to_dev(oh)))
    first = oh[:-1].copy()
    rnd = np.array([rng.integers(oh[k], oh[k + 1]) for k in range(256)])
    r_tr = _regret_stats(t, oh, best)
    r_un = _regret_stats(t, oh, best_u)
    r_fi = _regret_stats(t, oh, first)
    r_rn = _regret_stats(t, oh, rnd)
    say("mean regret: trained %.3f untrained %.3f first %.3f random %.3f" %
        (r_tr.mean(), r_un.mean(), r_fi.mean(), r_rn.mean()))
    say("median regret: trained %.3f untrained %.3f first %.3f random %.3f" %
        (np.median(r_tr), np.median(r_un), np.median(r_fi), np.median(r_rn)))
    assert last_loss < 0.2 * first_loss
    assert r_tr.mean() < 0.5 * min(r_un.mean(), r_fi.mean(), r_rn.mean())
    assert np.median(r_tr) < np.median(r_fi)


@pytest.mark.parametrize("precision,n", [("fp32", 16), ("fp32", 700), ("bf16", 16), ("bf16", 200),
                                         ("fp32", 2048)])
def test_backward_small_batches_match_oracle(precision, n):
    """Batches of one split (16, 200 and 700 rows: the weight gradients are
    written in place, no reduction) and of two (2048 rows), against the
    oracle's gradient of the same forward. fp32 must match to 1e-4. In bf16
    a rounding that flips a ReLU decision changes that row's contribution to
    a neuron's gradient entirely, one part in n of it, so the bound grows
    as the batch shrinks (measured 4e-2 at 16 rows, 2e-3 at 1500)."""
    widths = (32, 64, 128, 64, 32, 1)
    f, y, mu, sd = _batch(max(n, 600), 351)
    f, y = f[:n], y[:n]
    p = workload.he_init(widths, 352, bias_scale=0.1)
    m = adv.Model(widths, precision)
    m.set_params(p, mu, sd)
    yhat, saved = adv.advisor_mlp_forward(m.handle, to_dev(f))
    dy = (2.0 * (yhat.double() - to_dev(y)) / n).float()
    g = host(adv.advisor_mlp_backward(m.handle, dy, saved, n))
    x = oracle.normalize(f, mu, sd)
    _, g_ref = oracle.loss_grad(widths, p.astype(np.float64), x, y)
    err = _rel(g, g_ref)
    ew = _elementwise(g, g_ref, widths)
    say("backward %s n=%d: rel grad err %.2e, worst element %.2e" % (precision, n, err, ew))
    assert err <= (1e-4 if precision == "fp32" else (1e-1 if n < 100 else 3e-2))
    # element by element in bf16: one flipped ReLU decision changes a whole
    # row's product in a weight-gradient element; at 16 rows that one row can
    # be as large as the RMS of the matrix (measured 0.54 of it), at 700 rows
    # a small part of it (a transposed or misplaced element still gives
    # several times the RMS)
    assert ew <= (2e-3 if precision == "fp32" else (1.0 if n < 100 else 0.25))
