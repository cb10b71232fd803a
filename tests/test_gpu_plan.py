"""Captured plans (HIP graphs) replay exactly what the direct calls do.

Every replay is checked against the eager result, with eager work and
device synchronizations between the replays."""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, to_dev
from oracle import cost

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,widths", [("fp32", (32, 256, 256, 256, 1)),
                                              ("bf16", (32, 512, 512, 1)),
                                              ("fp8", (32, 256, 256, 1))])
def test_rank_plan_replays_match_eager(precision, widths):
    kd, vd, off = workload.make_descriptors(200, 8, 700, seed=501, invalid_frac=0.03)
    f, inv = oracle.featurize(kd, vd)
    mu, sd = oracle.zscore_fit(f[inv == 0])
    m = adv.Model(widths, precision)
    m.set_params(workload.he_init(widths, 502, bias_scale=0.1), mu, sd)
    if precision == "fp8":
        m.calibrate_fp8(to_dev(f[inv == 0][:4096]))
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    best_e, pred_e = m.rank(K, V, O, want_pred=True)
    best_e, pred_e = host(best_e), host(pred_e)
    best = torch.empty(off.size - 1, dtype=torch.int64, device="cuda")
    pred = torch.empty(vd.shape[0], dtype=torch.float32, device="cuda")
    plan = adv.Plan.rank(m, K, V, O, best, pred)
    for rep in range(3):
        best.fill_(-7)
        pred.fill_(123.0)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(best), best_e), rep
        assert np.array_equal(host(pred).view(np.int32), pred_e.view(np.int32)), rep
        # eager work between replays
        b2 = host(m.rank(K, V, O))
        assert np.array_equal(b2, best_e)
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_train_plan_replays_match_eager_steps(precision):
    widths = (32, 128, 128, 1)
    kd, vd, off = workload.make_descriptors(30, 64, 300, seed=511)
    f, inv = oracle.featurize(kd, vd)
    f = f[inv == 0][:5000]
    mu, sd = oracle.zscore_fit(f)
    y = cost.target(f, workload.noise(f.shape[0], 512))
    p0 = workload.he_init(widths, 513)
    F, Y = to_dev(f), to_dev(y)
    a = adv.Model(widths, precision)
    a.set_params(p0, mu, sd)
    b = adv.Model(widths, precision)
    b.set_params(p0, mu, sd)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    gn = torch.empty(1, dtype=torch.float64, device="cuda")
    plan = adv.Plan.train(b, F, Y, loss, gn, lr=2e-3)
    # creating the plan ran no step
    wb, _, _ = b.get_params()
    assert np.array_equal(wb, p0)
    for step in range(3):
        la, ga = adv.advisor_train_step(a.handle, F, Y, lr=2e-3)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        wa, _, _ = a.get_params()
        wb, _, _ = b.get_params()
        assert np.array_equal(wa.view(np.int32), wb.view(np.int32)), step
        assert host(la)[0] == host(loss)[0] and host(ga)[0] == host(gn)[0], step
        # eager predictions between replays
        m_pred = host(b.predict(F))
        assert np.isfinite(m_pred).all()
    _, _, t = adv.advisor_model_get_adam(b.handle)
    assert t == 3
    plan.close()
