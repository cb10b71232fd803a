"""The training step with section 5.3's optimizer (RMSprop, weight decay as
an L2 term, the RMSE loss of eq. rmse) against the float64 oracle: loss,
gradient and norm of one step, the update itself step by step with the
running average carried between calls, agreement with the MSE loss of the
Adam step, and the paper's recipe reaching its success bar (validation
NRMSE below 0.1) on synthetic runtimes."""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import elementwise_grad_err, host, say, to_dev
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


def _grads(m):
    g = torch.empty(m.param_count, dtype=torch.float32, device="cuda")
    adv.advisor_model_grads(m.handle, g)
    return host(g)


@pytest.mark.parametrize("loss", ["rmse", "mse"])
def test_rmsprop_step_fp32_matches_oracle(loss):
    widths = (32, 256, 256, 256, 1)
    f, y, mu, sd = _batch(3000, 411)
    p = workload.he_init(widths, 412, bias_scale=0.1)
    m = adv.Model(widths, "fp32")
    m.set_params(p, mu, sd)
    lo, gn = adv.advisor_train_step_rmsprop(m.handle, to_dev(f), to_dev(y), lr=1e-2, alpha=0.99,
                                            eps=1e-8, weight_decay=1e-4, loss=loss)
    lo, gn = host(lo)[0], host(gn)[0]
    g = _grads(m)
    w_new, _, _ = m.get_params()
    _, v_gpu, t = adv.advisor_model_get_adam(m.handle)
    x = oracle.normalize(f, mu, sd)
    p64 = p.astype(np.float64)
    if loss == "rmse":
        l_ref, g_ref = oracle.rmse_loss_grad(widths, p64, x, y)
    else:
        l_ref, g_ref = oracle.loss_grad(widths, p64, x, y)
    say("rmsprop %s: loss %.6f ref %.6f, rel grad err %.2e" % (loss, lo, l_ref, _rel(g, g_ref)))
    assert abs(lo - l_ref) / l_ref <= 1e-5
    assert _rel(g, g_ref) <= 1e-4
    assert elementwise_grad_err(g, g_ref, widths) <= 2e-3
    assert abs(gn - np.linalg.norm(g.astype(np.float64))) <= 1e-6 * gn
    assert t == 0  # Adam's step count is not RMSprop's business
    # the update, in float64 on the gradient the GPU used
    w = p64.copy()
    v = np.zeros_like(w)
    oracle.rmsprop(w, v, g.astype(np.float64), lr=1e-2, alpha=0.99, eps=1e-8, weight_decay=1e-4)
    assert np.allclose(v_gpu, v, rtol=1e-5, atol=1e-30)
    step, ref = w_new.astype(np.float64) - p64, w - p64
    gd = np.abs(g.astype(np.float64) + 1e-4 * p64)
    big = gd > 1e-3 * gd.max()
    assert np.allclose(step[big], ref[big], rtol=1e-4, atol=1e-8)
    assert np.max(np.abs(step - ref)) <= 0.1 * 2e-2  # every step is at most lr / sqrt(1 - alpha)


def test_rmsprop_mse_loss_equals_adam_step_loss():
    """Same parameters and batch: the MSE the RMSprop step reports is the
    Adam step's, bit for bit (same forward, same float64 summation)."""
    widths = (32, 128, 128, 1)
    f, y, mu, sd = _batch(2500, 421)
    p = workload.he_init(widths, 422)
    a = adv.Model(widths, "fp32")
    a.set_params(p, mu, sd)
    b = adv.Model(widths, "fp32")
    b.set_params(p, mu, sd)
    la, ga = adv.advisor_train_step(a.handle, to_dev(f), to_dev(y))
    lb, gb = adv.advisor_train_step_rmsprop(b.handle, to_dev(f), to_dev(y), loss="mse")
    assert host(la)[0] == host(lb)[0]
    assert host(ga)[0] == host(gb)[0]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_rmsprop_updates_carry_running_average(precision):
    """Four steps: after each, the new master weights equal the oracle's
    RMSprop applied to the weights before it, the gradient the GPU used, and
    the running average carried from the previous steps."""
    widths = (32, 64, 64, 1)
    f, y, mu, sd = _batch(1500, 431)
    p = workload.he_init(widths, 432, bias_scale=0.1)
    m = adv.Model(widths, precision)
    m.set_params(p, mu, sd)
    F, Y = to_dev(f), to_dev(y)
    w = p.astype(np.float64)
    v = np.zeros_like(w)
    for k in range(4):
        adv.advisor_train_step_rmsprop(m.handle, F, Y, lr=3e-3, weight_decay=1e-4)
        g = _grads(m).astype(np.float64)
        w_gpu, _, _ = m.get_params()
        w_prev = w.copy()
        oracle.rmsprop(w, v, g, lr=3e-3, alpha=0.99, eps=1e-8, weight_decay=1e-4)
        step_gpu = w_gpu.astype(np.float64) - w_prev
        step_ref = w - w_prev
        err = np.max(np.abs(step_gpu - step_ref))
        say("%s step %d: max |step - ref| %.2e (lr 3e-3)" % (precision, k, err))
        # fp32 rounding of g', v and w: far below the step size lr / sqrt(1 - alpha)
        assert err <= 1e-6
        w = w_gpu.astype(np.float64)  # follow the GPU's (fp32-rounded) weights


def test_rmsprop_recipe_reaches_nrmse_bar():
    """Section 5.3's recipe (RMSprop, weight decay 1e-4, RMSE loss, lr 0.01
    stepped down 10x every 30 epochs, an 80/20 split, Z-score inputs) on
    synthetic runtimes of the same form: the validation NRMSE ends below
    the paper's 0.1 success bar, and every epoch's schedule is the paper's.
    Batches of 256 rows keep the test short (the paper uses 16)."""
    widths = (32, 64, 128, 64, 32, 1)
    f, y, _, _ = _batch(20000, 441)
    n_train = int(0.8 * f.shape[0])
    mu, sd = oracle.zscore_fit(f[:n_train])
    m = adv.Model(widths, "fp32")
    m.set_params(workload.he_init(widths, 442), mu, sd)
    tr = adv.RMSpropTrainer(m)
    F, Y = to_dev(f[:n_train]), to_dev(y[:n_train])
    bs = 256
    rng = np.random.default_rng(443)
    losses = []
    for epoch in range(40):
        tr.set_epoch(epoch)
        assert tr.lr == oracle.step_lr(epoch)
        perm = to_dev(rng.permutation(n_train))
        last = None
        for s in range(0, n_train - bs + 1, bs):
            idx = perm[s:s + bs]
            last, _ = tr.step(F[idx].contiguous(), Y[idx].contiguous())
        losses.append(host(last)[0])
    pred = host(m.predict(to_dev(f[n_train:])))
    yv = y[n_train:]
    rmse = oracle.rmse(pred.astype(np.float64), yv)
    nrmse = oracle.nrmse(pred.astype(np.float64), yv)
    say("recipe: train RMSE %.3f -> %.3f, validation RMSE %.3f NRMSE %.4f" %
        (losses[0], losses[-1], rmse, nrmse))
    assert losses[-1] < losses[0]
    assert nrmse < 0.1


def test_paper_recipe_one_model_batch16():
    """Section 5.3's recipe as written for one target, with eager library
    steps (no captured plan): 2000 synthetic runtimes of 200 kernels,
    32-64-128-64-32-1 with Glorot weights and zero biases, an 80/20 split,
    Z-score inputs, batches of 16, 150 epochs of RMSprop (lr 0.01 divided by
    10 every 30 epochs, weight decay 1e-4) on the RMSE loss: 15,000 steps.
    The validation NRMSE ends below the paper's 0.1 bar."""
    widths = (32, 64, 128, 64, 32, 1)
    N, bs, epochs = 2000, 16, 150
    n_train = int(0.8 * N)
    kd, vd, off = workload.make_descriptors(200, 8, 40, 480)
    f, inv = oracle.featurize(kd, vd)
    f = f[inv == 0]
    f = f[np.random.default_rng(482).permutation(f.shape[0])[:N]]
    y = cost.target(f, workload.noise(f.shape[0], 483))
    mu, sd = oracle.zscore_fit(f[:n_train])
    m = adv.Model(widths, "fp32")
    m.set_params(workload.glorot_init(widths, 481), mu, sd)
    tr = adv.RMSpropTrainer(m)
    F, Y = to_dev(f[:n_train]), to_dev(y[:n_train])
    rng = np.random.default_rng(489)
    first = last = None
    for epoch in range(epochs):
        tr.set_epoch(epoch)
        assert tr.lr == oracle.step_lr(epoch)
        perm = to_dev(rng.permutation(n_train))
        for s in range(0, n_train - bs + 1, bs):
            idx = perm[s:s + bs]
            last, _ = tr.step(F[idx].contiguous(), Y[idx].contiguous())
        if first is None:
            first = host(last)[0]
        if epoch % 30 == 29:
            say("recipe, one model, batch 16: epoch %d, batch RMSE %.3f" % (epoch, host(last)[0]))
    pred = host(m.predict(to_dev(f[n_train:]))).astype(np.float64)
    nr = oracle.nrmse(pred, y[n_train:])
    say("recipe, one model, batch 16: batch RMSE %.3f -> %.3f, validation NRMSE %.4f"
        % (first, host(last)[0], nr))
    assert nr < 0.1
    m.close()


@pytest.mark.parametrize("precision,n", [("fp32", 16), ("bf16", 3000)])
def test_rmsprop_plan_replays_match_eager_steps(precision, n):
    """A captured RMSprop step (the paper's batch of 16 rows, and a larger
    one) replays exactly the eager step, with eager work and device
    synchronizations between replays; the eager and replayed step times at
    batch 16 are printed."""
    import time
    widths = (32, 64, 128, 64, 32, 1)
    f, y, mu, sd = _batch(max(n, 600), 451)
    f, y = f[:n], y[:n]
    p0 = workload.he_init(widths, 452)
    F, Y = to_dev(f), to_dev(y)
    a = adv.Model(widths, precision)
    a.set_params(p0, mu, sd)
    b = adv.Model(widths, precision)
    b.set_params(p0, mu, sd)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    gn = torch.empty(1, dtype=torch.float64, device="cuda")
    plan = adv.Plan.train_rmsprop(b, F, Y, loss, gn, lr=1e-2, weight_decay=1e-4)
    wb, _, _ = b.get_params()
    assert np.array_equal(wb, p0)  # creating the plan ran no step
    for step in range(3):
        la, ga = adv.advisor_train_step_rmsprop(a.handle, F, Y, lr=1e-2, weight_decay=1e-4)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        wa, _, _ = a.get_params()
        wb, _, _ = b.get_params()
        assert np.array_equal(wa.view(np.int32), wb.view(np.int32)), step
        assert host(la)[0] == host(loss)[0] and host(ga)[0] == host(gn)[0], step
        assert np.isfinite(host(b.predict(F))).all()
    if n == 16:
        reps = 200
        for name, fn in (("eager", lambda: adv.advisor_train_step_rmsprop(
                a.handle, F, Y, lr=1e-2, weight_decay=1e-4, loss_out=loss, gnorm_out=gn)),
                         ("plan", plan.launch)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            say("batch-16 RMSprop step, %s: %.1f us" % (name, (time.perf_counter() - t0) / reps * 1e6))
    plan.close()


def test_multi_model_plan_matches_separate_steps():
    """Seven models of the paper's shape (one per cluster of its experiments),
    each with its own 16-row batch, stepped together by one plan: every
    replay leaves each model exactly as its own eager step does. The replay
    time is printed beside seven single-model plans."""
    import time
    widths = (32, 64, 128, 64, 32, 1)
    T = 7
    eager, planned, feats, ys = [], [], [], []
    for t in range(T):
        f, y, mu, sd = _batch(600, 460 + t)
        f, y = f[:16], y[:16]
        p0 = workload.he_init(widths, 470 + t)
        a = adv.Model(widths, "fp32")
        a.set_params(p0, mu, sd)
        b = adv.Model(widths, "fp32")
        b.set_params(p0, mu, sd)
        eager.append(a)
        planned.append(b)
        feats.append(to_dev(f))
        ys.append(to_dev(y))
    loss = torch.zeros(T, dtype=torch.float64, device="cuda")
    gn = torch.zeros(T, dtype=torch.float64, device="cuda")
    plan = adv.Plan.train_rmsprop_multi(planned, feats, ys, loss, gn)
    for step in range(3):
        ref = []
        for t in range(T):
            la, ga = adv.advisor_train_step_rmsprop(eager[t].handle, feats[t], ys[t])
            ref.append((host(la)[0], host(ga)[0]))
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        lo, gg = host(loss), host(gn)
        for t in range(T):
            wa, _, _ = eager[t].get_params()
            wb, _, _ = planned[t].get_params()
            assert np.array_equal(wa.view(np.int32), wb.view(np.int32)), (step, t)
            assert lo[t] == ref[t][0] and gg[t] == ref[t][1], (step, t)
        assert np.isfinite(host(planned[0].predict(feats[0]))).all()
    singles = [adv.Plan.train_rmsprop(eager[t], feats[t], ys[t], loss[t:t + 1], gn[t:t + 1])
               for t in range(T)]
    reps = 50
    for name, fn in (("one plan for all 7", plan.launch),
                     ("7 single-model plans", lambda: [s.launch() for s in singles])):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        say("7 models x 16 rows, %s: %.1f us per step of all" %
            (name, (time.perf_counter() - t0) / reps * 1e6))
    for s in singles:
        s.close()
    plan.close()


def test_paper_recipe_seven_models_batch16_eager():
    """Section 5.3's recipe for seven targets (one model per cluster of the
    paper's experiments, each on 2000 synthetic runtimes of 200 kernels of
    its own), trained together with eager library steps: per minibatch of 16
    rows every model takes its RMSprop step (lr 0.01 divided by 10 every 30
    epochs, weight decay 1e-4, RMSE loss), 150 epochs each, 105,000 steps in
    all. Every model's validation NRMSE ends below the paper's 0.1 bar. The
    same recipe through one captured plan of the seven steps is the skipped
    test below."""
    widths = (32, 64, 128, 64, 32, 1)
    T, N, bs, epochs = 7, 2000, 16, 150
    n_train = int(0.8 * N)
    models, trainers, data = [], [], []
    for t in range(T):
        kd, vd, off = workload.make_descriptors(200, 8, 40, 480 + 10 * t)
        f, inv = oracle.featurize(kd, vd)
        f = f[inv == 0]
        f = f[np.random.default_rng(482 + 10 * t).permutation(f.shape[0])[:N]]
        y = cost.target(f, workload.noise(f.shape[0], 483 + 10 * t))
        mu, sd = oracle.zscore_fit(f[:n_train])
        m = adv.Model(widths, "fp32")
        m.set_params(workload.glorot_init(widths, 481 + 10 * t), mu, sd)
        models.append(m)
        trainers.append(adv.RMSpropTrainer(m))
        data.append((to_dev(f[:n_train]), to_dev(y[:n_train]), f[n_train:], y[n_train:]))
    rng = np.random.default_rng(489)
    first, last = None, [None] * T
    for epoch in range(epochs):
        for tr in trainers:
            tr.set_epoch(epoch)
        # each model's epoch order, gathered once: its batches are row slices
        order = [to_dev(rng.permutation(n_train)) for _ in range(T)]
        Fe = [data[t][0][order[t]] for t in range(T)]
        Ye = [data[t][1][order[t]] for t in range(T)]
        for s in range(0, n_train - bs + 1, bs):
            for t in range(T):
                last[t], _ = trainers[t].step(Fe[t][s:s + bs], Ye[t][s:s + bs])
        if first is None:
            first = [host(v)[0] for v in last]
        if epoch % 30 == 29:
            say("recipe, seven models, batch 16: epoch %d" % epoch)
    for t in range(T):
        pred = host(models[t].predict(to_dev(data[t][2]))).astype(np.float64)
        nr = oracle.nrmse(pred, data[t][3])
        say("model %d: batch RMSE %.3f -> %.3f, validation NRMSE %.4f"
            % (t, first[t], host(last[t])[0], nr))
        assert nr < 0.1
    for m in models:
        m.close()


@pytest.mark.skip(reason="crashed the host inside hipGraphLaunch twice (a segmentation fault "
                         "during thousands of unsynchronized replays of the seven-model plan, "
                         "then in the full suite after the destroy fix); kept off the GPU until "
                         "the cause is shown")
def test_paper_recipe_seven_models_batch16():
    """Section 5.3's recipe as written, for seven models at once (one per
    cluster of the paper's experiments, each on 2000 synthetic runtimes of
    200 kernels):
    32-64-128-64-32-1 (the paper's multiples of the input count), Glorot
    weights and zero biases, batches of 16, 150 epochs of RMSprop with lr
    0.01 divided by 10 every 30 epochs and weight decay 1e-4, the RMSE loss,
    an 80/20 split and Z-score inputs. Each epoch's minibatches are gathered
    into the plan's fixed buffers and the plan (the seven models' steps in
    one branch; it held one graph branch per model, forked onto a stream of
    its own each, when the host crashed) is rebuilt when the learning rate
    steps. Every model's validation NRMSE ends below the paper's 0.1 bar."""
    widths = (32, 64, 128, 64, 32, 1)
    T, N, bs, epochs = 7, 2000, 16, 150
    n_train = int(0.8 * N)
    models, data = [], []
    for t in range(T):
        # 2000 variants of 200 kernels, shuffled before the 80/20 split
        kd, vd, off = workload.make_descriptors(200, 8, 40, 480 + 10 * t)
        f, inv = oracle.featurize(kd, vd)
        f = f[inv == 0]
        f = f[np.random.default_rng(482 + 10 * t).permutation(f.shape[0])[:N]]
        y = cost.target(f, workload.noise(f.shape[0], 483 + 10 * t))
        mu, sd = oracle.zscore_fit(f[:n_train])
        m = adv.Model(widths, "fp32")
        m.set_params(workload.glorot_init(widths, 481 + 10 * t), mu, sd)
        models.append(m)
        data.append((to_dev(f[:n_train]), to_dev(y[:n_train]), f[n_train:], y[n_train:]))
    fb = [torch.empty((bs, 32), dtype=torch.int64, device="cuda") for _ in range(T)]
    yb = [torch.empty(bs, dtype=torch.float64, device="cuda") for _ in range(T)]
    loss = torch.zeros(T, dtype=torch.float64, device="cuda")
    gn = torch.zeros(T, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(489)
    plan, plan_lr = None, None
    first = None
    for epoch in range(epochs):
        lr = adv.step_lr(epoch)
        assert lr == oracle.step_lr(epoch)
        if lr != plan_lr:
            if plan is not None:
                torch.cuda.synchronize()
                plan.close()
            plan = adv.Plan.train_rmsprop_multi(models, fb, yb, loss, gn, lr=lr)
            plan_lr = lr
        perms = [to_dev(rng.permutation(n_train)) for _ in range(T)]
        for s in range(0, n_train - bs + 1, bs):
            for t in range(T):
                idx = perms[t][s:s + bs]
                torch.index_select(data[t][0], 0, idx, out=fb[t])
                torch.index_select(data[t][1], 0, idx, out=yb[t])
            plan.launch()
        if first is None:
            first = host(loss).copy()
    torch.cuda.synchronize()
    plan.close()
    last = host(loss)
    for t in range(T):
        pred = host(models[t].predict(to_dev(data[t][2]))).astype(np.float64)
        nr = oracle.nrmse(pred, data[t][3])
        say("model %d: batch RMSE %.3f -> %.3f, validation NRMSE %.4f" % (t, first[t], last[t], nr))
        assert nr < 0.1
