"""Throughput of the cost-model hot path on one MI355X.

One step = one advisor_rank call over the whole synthetic workload: feature
extraction of every variant, Z-score, the MLP on the matrix cores and the
per-kernel argmin (the paper's prediction flow, many kernels at once),
replayed from a HIP graph with the tile shape the library's autotuner chose.
The descriptors and weights are resident in HBM before the timed region; the
timed region is exactly --steps replays bracketed by device synchronization.

Prints one JSON line. `value` is variants ranked per second; `roofline`
prices the fused tile kernel (the dominant kernel) against the matrix-core
peak of its precision, with its duration taken from HIP events recorded
around each of its launches; `cpu_baseline` is the float64 CPU oracle timed
on a seeded sample of whole kernels of the same workload on this host.
`precisions` repeats the measurement for the other compute precisions on the
same inputs, each with its argmin agreement against the oracle on the sample
(He-initialized weights) and for a network first trained by the library on
the synthetic runtime model.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workload  # noqa: E402

# MI355X published dense peaks (TFLOP/s) and HBM bandwidth (GB/s)
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}
PEAK_HBM_GBS = 8000.0
DEFAULT_PRECISION = {1: "fp32", 2: "fp32", 3: "bf16", 5: "fp8"}
DEFAULT_ALSO = {1: "", 2: "bf16", 3: "fp32", 5: "bf16,fp32"}
WORKLOAD_NAME = {
    1: "single kernel x 256 variants, 32-64-64-1",
    2: "4096 kernels x U[16,1024] variants (2.1M), 32-256x3-1",
    3: "16384 kernels x U[64,1024] variants (8.9M), 32-512x4-1",
    5: "32768 kernels x U[128,1024] variants (18.9M), 32-1024x4-1",
}
PROFILE_DIR = os.path.join(ROOT, "profiles")


def layer_flops(widths):
    return [2 * widths[i] * widths[i + 1] for i in range(len(widths) - 1)]


def roofline_peak(widths, precision):
    """Peak for the whole network: the fp8 model keeps its first layer in
    bf16, so its roofline time is the sum of per-layer times."""
    fl = layer_flops(widths)
    if precision != "fp8":
        return PEAK_TFLOPS[precision]
    t = fl[0] / PEAK_TFLOPS["bf16"] + sum(fl[1:-1]) / PEAK_TFLOPS["fp8"] + fl[-1] / PEAK_TFLOPS["bf16"]
    return sum(fl) / t


def kernel_source_hash():
    """Hash of the sources of the fused tile kernel and its launch shapes; a
    stored traffic measurement only applies to the kernel it was taken on."""
    h = hashlib.sha256()
    for f in ("mlp_tile.h", "features.h", "mlp.hip"):
        with open(os.path.join(ROOT, "paper_2301_03636_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(cfg, precision):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE, scaled by a copy-kernel calibration), if taken on the
    current kernel sources; else None."""
    path = os.path.join(PROFILE_DIR, "traffic_tiles_cfg%d_%s.json" % (cfg, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def make_inputs(cfg, seed_desc=None):
    c = workload.WORKLOADS[cfg]
    s = workload.seeds(cfg)
    kd, vd, off = workload.make_descriptors(c["n_kernels"], c["count_lo"], c["count_hi"],
                                            s["desc"] if seed_desc is None else seed_desc)
    params = workload.he_init(c["widths"], s["w"])
    return kd, vd, off, params, tuple(c["widths"])


def time_rank(adv, torch, model, kdd, vdd, offd, best, steps, warmup):
    """Two timed regions of `steps` calls each. First the fused kernel's own
    duration: eager advisor_rank calls with HIP events recorded around each
    tile-kernel launch on its stream. Then the step time: replays of the
    call captured into a HIP graph, bracketed by device synchronization."""
    for _ in range(warmup):
        model.rank(kdd, vdd, offd, best_out=best)
    torch.cuda.synchronize()
    adv.advisor_profile_enable(True)
    for _ in range(steps):
        model.rank(kdd, vdd, offd, best_out=best)
    torch.cuda.synchronize()
    launches, kern_ms = adv.advisor_profile_read()
    adv.advisor_profile_enable(False)
    plan = adv.Plan.rank(model, kdd, vdd, offd, best)
    for _ in range(warmup):
        plan.launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        plan.launch()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.close()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    pct = {"p10": float(np.percentile(per, 10)), "p50": float(np.percentile(per, 50)),
           "p90": float(np.percentile(per, 90))}
    return (t1 - t0) * 1e3 / steps, kern_ms / max(launches, 1), launches, pct


def time_with_transfers(adv, torch, model, kd, vd, off, kdd, vdd, offd, best, steps, warmup):
    """The same ranking with the descriptors handed over in pinned host
    memory: each step copies kdesc, vdesc and offsets to the device, ranks
    (graph replay) and copies `best` back, all on one stream."""
    pin = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (kd, vd, off)]
    best_h = torch.empty(best.shape, dtype=best.dtype).pin_memory()
    plan = adv.Plan.rank(model, kdd, vdd, offd, best)

    def step():
        for dev, host in zip((kdd, vdd, offd), pin):
            dev.copy_(host, non_blocking=True)
        plan.launch()
        best_h.copy_(best, non_blocking=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for dev, host in zip((kdd, vdd, offd), pin):
        dev.copy_(host, non_blocking=True)
    e[1].record()
    best_h.copy_(best, non_blocking=True)
    e[2].record()
    torch.cuda.synchronize()
    plan.close()
    h2d_bytes = sum(int(a.nbytes) for a in (kd, vd, off))
    h2d_ms, d2h_ms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    return {"ms_per_step": ms, "value": vd.shape[0] / (ms / 1e3), "h2d_bytes": h2d_bytes,
            "h2d_ms": h2d_ms, "h2d_gbs": h2d_bytes / (h2d_ms / 1e3) / 1e9, "d2h_ms": d2h_ms}


def stage_kernels(adv, torch, kdd, vdd, offd, steps):
    """advisor_featurize and advisor_rank_preds alone on the workload, each
    priced against HBM bandwidth with its algorithmic bytes: featurize reads
    64 B of vdesc per variant (kdesc rows are amortized over a kernel's
    variants: 128 B per kernel) and writes 256 B of features and a 1-byte
    flag; the argmin reads a 4-byte prediction per variant and 8 B of
    offsets and writes 8 B of `best` per kernel; the top-10 list reads the
    same and writes 10 x (8 B index + 4 B prediction) per kernel."""
    nv, nk = vdd.shape[0], offd.shape[0] - 1
    feat = torch.empty((nv, 32), dtype=torch.int64, device=vdd.device)
    inv = torch.empty(nv, dtype=torch.uint8, device=vdd.device)
    pred = torch.empty(nv, dtype=torch.float32, device=vdd.device).normal_()
    best = torch.empty(nk, dtype=torch.int64, device=vdd.device)
    tidx = torch.empty((nk, 10), dtype=torch.int64, device=vdd.device)
    tval = torch.empty((nk, 10), dtype=torch.float32, device=vdd.device)
    out = {}
    for name, fn, nbytes in (
            ("featurize", lambda: adv.advisor_featurize(kdd, vdd, feat_out=feat, invalid_out=inv),
             nv * (64 + 256 + 1) + nk * 128),
            ("rank_preds", lambda: adv.advisor_rank_preds(pred, offd, best_out=best),
             nv * 4 + nk * 16 + 8),
            ("topn10_preds", lambda: adv.advisor_topn_preds(pred, offd, 10, idx_out=tidx,
                                                            val_out=tval),
             nv * 4 + nk * (8 + 10 * 12) + 8)):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        gbs = nbytes / (ms / 1e3) / 1e9
        out[name] = {"ms": ms, "bytes": nbytes, "achieved_gbs": gbs, "peak_gbs": PEAK_HBM_GBS,
                     "frac": gbs / PEAK_HBM_GBS}
    del feat, inv, pred, best, tidx, tval
    # the method's integer steps on synthetic inputs of their own: variant
    # generation for 262,144 kernels of 1-4 loops (8 B of loop count read per
    # kernel, 8 B of offsets and 48 B per variant row written), and the data
    # analysis of 4 variables per kernel for 1,048,576 kernels (1 B of access
    # bits and 8 B of size read and 1 B of class written per variable, 8 B of
    # offsets read and 24 B of byte totals written per kernel)
    g = torch.Generator(device="cpu").manual_seed(77)
    nk_v = 1 << 18
    nl = torch.randint(1, 5, (nk_v,), generator=g, dtype=torch.int64).to(vdd.device)
    offv = adv.advisor_count_variants(nl)
    nv_v = int(offv[-1].item())
    rows = torch.empty((nv_v, 6), dtype=torch.int64, device=vdd.device)
    nk_d = 1 << 20
    acc = torch.randint(0, 32, (4 * nk_d,), generator=g, dtype=torch.uint8).to(vdd.device)
    nbytes = torch.randint(0, 1 << 30, (4 * nk_d,), generator=g, dtype=torch.int64).to(vdd.device)
    offd_d = torch.arange(0, 4 * nk_d + 1, 4, dtype=torch.int64, device=vdd.device)
    for name, fn, nbytes_alg in (
            ("variant_generation", lambda: adv.advisor_enumerate_variants(
                nl, 7, offsets=adv.advisor_count_variants(nl, 7, offsets_out=offv),
                variants_out=rows), nk_v * 16 + nv_v * 48 + 8),
            ("data_analysis", lambda: adv.advisor_classify_maps(acc, nbytes, offd_d),
             4 * nk_d * 10 + nk_d * 32 + 8)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        gbs = nbytes_alg / (ms / 1e3) / 1e9
        out[name] = {"ms": ms, "bytes": nbytes_alg, "achieved_gbs": gbs, "peak_gbs": PEAK_HBM_GBS,
                     "frac": gbs / PEAK_HBM_GBS,
                     "units": {"variant_generation": "%d kernels, %d variants" % (nk_v, nv_v),
                               "data_analysis": "%d kernels x 4 variables" % nk_d}[name]}
    del nl, offv, rows, acc, nbytes, offd_d
    return out


def cpu_baseline_leg(kd, vd, off, widths, params, mu, sd, seconds, gpu_best_by_prec):
    """The float64 oracle (as written, parallel over kernels) on a seeded
    sample of whole kernels sized to about `seconds` of CPU time."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    p64 = params.astype(np.float64)

    def run(n_kernels, seed):
        ks, rows, sub_off = workload.sample_kernels(off, n_kernels, seed)
        vsub = vd[rows].copy()
        vsub[:, 0] = np.repeat(np.arange(ks.size), sub_off[1:] - sub_off[:-1])
        t0 = time.perf_counter()
        best, _ = oracle.rank(kd[ks], vsub, sub_off, widths, p64, mu, sd, n_threads=threads,
                              want_pred=False)
        dt = time.perf_counter() - t0
        glob = np.where(best >= 0, rows[np.maximum(best, 0)], -1)
        return ks, rows.size, dt, glob

    nk = off.size - 1
    probe = min(nk, max(1, 2 * threads))
    _, nv_probe, dt_probe, _ = run(probe, 4242)
    per_variant = dt_probe / max(nv_probe, 1)
    avg = (off[-1] / nk)
    n_sample = int(min(nk, max(probe, seconds / max(per_variant * avg, 1e-9))))
    ks, nv_s, dt, best_cpu = run(n_sample, 4243)
    agree = {}
    for prec, gb in gpu_best_by_prec.items():
        agree[prec] = float(np.mean(gb[ks] == best_cpu))
    return {
        "value": nv_s / dt,
        "unit": "variants/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d of %d kernels (seeded), %d variants, %.1f s wall" % (ks.size, nk, nv_s, dt),
    }, agree, per_variant


def trained_agreement(adv, torch, to_dev, kd, vd, off, widths, precs, per_variant, seconds,
                      refine_k):
    """Argmin agreement with the oracle for a network trained by the
    library's own training step on the synthetic runtime model (the targets
    of the gain test), which is what a user of the method ranks with. A
    trained network predicts near-equal runtimes for variants whose true
    runtimes are near-equal (e.g. launch shapes of a memory-bound kernel), so
    lower-precision picks can differ from the float64 pick among near-ties;
    the gap between the two picks under the oracle's own prediction says
    what such a disagreement costs."""
    import oracle
    from oracle import cost
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    rows = workload.sample_rows(vd.shape[0], 131072, 4300)
    f, inv = oracle.featurize(kd, vd[rows])
    f = f[inv == 0]
    mu, sd = oracle.zscore_fit(f)
    y = cost.target(f, workload.noise(f.shape[0], 4301))
    m = adv.Model(widths, "bf16")
    m.set_params(workload.he_init(widths, 4302), mu, sd)
    F, Y = to_dev(f), to_dev(y)
    rng = np.random.default_rng(4303)
    loss = None
    for _ in range(400):
        idx = torch.from_numpy(rng.integers(0, f.shape[0], 8192)).to(F.device)
        loss, _ = adv.advisor_train_step(m.handle, F[idx].contiguous(), Y[idx].contiguous(),
                                         lr=2e-3)
    w, _, _ = m.get_params()
    final_loss = float(loss.item())
    m.close()
    nk = off.size - 1
    n_sample = int(min(nk, max(8, seconds / max(per_variant * (off[-1] / nk), 1e-9))))
    ks, rws, sub_off = workload.sample_kernels(off, n_sample, 4304)
    vsub = vd[rws].copy()
    vsub[:, 0] = np.repeat(np.arange(ks.size), sub_off[1:] - sub_off[:-1])
    best_cpu, pred_cpu = oracle.rank(kd[ks], vsub, sub_off, widths, w.astype(np.float64), mu,
                                     sd, n_threads=threads, want_pred=True)
    K, V, O = to_dev(kd[ks]), to_dev(vsub), to_dev(sub_off)
    agree, regret = {}, {}
    has = best_cpu >= 0
    hi = adv.Model(widths, "fp32")
    hi.set_params(w, mu, sd)
    for p in precs:
        g = adv.Model(widths, p)
        g.set_params(w, mu, sd)
        if p == "fp8":
            g.calibrate_fp8(F)
        picks = {p: g.rank(K, V, O).cpu().numpy()}
        rk = refine_k_for(p, refine_k)
        if p != "fp32" and rk > 0:
            picks[p + "_refined"] = g.rank_refined(hi, K, V, O, top_k=rk).cpu().numpy()
            if p == "fp8":
                mid = adv.Model(widths, "bf16")
                mid.set_params(w, mu, sd)
                picks["fp8_refined_bf16"] = g.rank_refined(mid, K, V, O, top_k=rk).cpu().numpy()
                mid.close()
        g.close()
        for name, best_gpu in picks.items():
            agree[name] = float(np.mean(best_gpu == best_cpu))
            # how much worse the GPU's pick is by the oracle's own prediction
            # (ln us): a disagreement between near-tied variants costs ~0
            gap = pred_cpu[best_gpu[has]] - pred_cpu[best_cpu[has]]
            regret[name] = {"mean": float(gap.mean()), "max": float(gap.max()),
                            "frac_below_0.01": float(np.mean(gap < 0.01))}
    hi.close()
    return agree, {"train_steps": 400, "batch": 8192, "final_loss": final_loss,
                   "sample_kernels": int(ks.size), "sample_variants": int(rws.size),
                   "pick_gap_ln_us_by_oracle_prediction": regret,
                   "top2_gap_ln_us_histogram": top2_gap_histogram(pred_cpu, best_cpu, sub_off)}


def top2_gap_histogram(pred, best, off):
    """Per kernel, the oracle's margin between its best and second-best
    variant (ln us): how many kernels a low-precision ranking can only get
    right by resolving a near-tie. Counts per bin [lo, hi)."""
    edges = [0.0, 1e-6, 1e-4, 1e-3, 1e-2, 1e-1, np.inf]
    gaps = []
    for k in range(off.size - 1):
        if best[k] < 0 or off[k + 1] - off[k] < 2:
            continue
        seg = pred[off[k]:off[k + 1]]
        seg = seg[np.isfinite(seg)]
        if seg.size < 2:
            continue
        two = np.partition(seg, 1)[:2]
        gaps.append(float(two[1] - two[0]))
    counts, _ = np.histogram(np.asarray(gaps), bins=edges)
    names = ["0", "<1e-6", "<1e-4", "<1e-3", "<1e-2", "<1e-1", ">=1e-1"]
    exact0 = int(np.sum(np.asarray(gaps) == 0.0))
    out = {"exact_tie": exact0}
    out.update({n: int(c) for n, c in zip(names[1:], counts)})
    out["<1e-6"] -= exact0  # the first bin [0, 1e-6) includes the exact ties
    return out


def refine_k_for(precision, requested):
    """Candidates per kernel for the fp32 re-ranking: 8 after bf16, 16 after
    fp8 (fp8's 3-bit mantissas scatter near-tied predictions further)."""
    if requested is not None:
        return requested
    return {"bf16": 8, "fp8": 16}.get(precision, 0)


def train_flops_per_sample(widths):
    """Forward, input gradients of every layer but the first, and weight
    gradients of every layer: 2 flops per multiply-add."""
    fl = layer_flops(widths)
    return sum(fl) + sum(fl[1:]) + sum(fl)


def train_leg(adv, torch, d, steps, warmup):
    """Training throughput: batch 65536 of the 4096-kernel workload, bf16
    32-512x4-1, Adam lr 1e-3, float64 loss and gradient norm. The targets are
    seeded draws of the same scale as ln(runtime in us) (the timing does not
    depend on their values; the tests train on the synthetic runtime model)."""
    c = workload.WORKLOADS[4]
    s = workload.seeds(4)
    widths = tuple(c["widths"])
    B = c["batch"]
    kd, vd, off = workload.make_descriptors(c["n_kernels"], c["count_lo"], c["count_hi"], s["desc"])
    rows = workload.sample_rows(vd.shape[0], B, s["desc"] + 11)
    feat, inv = adv.advisor_featurize(torch.from_numpy(kd).to(d), torch.from_numpy(vd[rows]).to(d))
    assert int(inv.sum().item()) == 0
    mu, sd = adv.advisor_zscore_fit(feat)
    y = torch.from_numpy(10.0 + 3.0 * workload.noise(B, s["noise"])).to(d)
    m = adv.Model(widths, "bf16")
    m.set_params(workload.he_init(widths, s["w"]), mu.cpu().numpy(), sd.cpu().numpy())
    loss = torch.empty(1, dtype=torch.float64, device=d)
    gn = torch.empty(1, dtype=torch.float64, device=d)
    for _ in range(warmup):
        adv.advisor_train_step(m.handle, feat, y, 1e-3, 0.9, 0.999, 1e-8, loss, gn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        adv.advisor_train_step(m.handle, feat, y, 1e-3, 0.9, 0.999, 1e-8, loss, gn)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    loss_adam = float(loss.item())
    # the paper's optimizer on the same batch (RMSprop, weight decay, RMSE loss)
    for _ in range(max(1, warmup)):
        adv.advisor_train_step_rmsprop(m.handle, feat, y, 1e-3, 0.99, 1e-8, 1e-4, "rmse", loss, gn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        adv.advisor_train_step_rmsprop(m.handle, feat, y, 1e-3, 0.99, 1e-8, 1e-4, "rmse", loss, gn)
    torch.cuda.synchronize()
    ms_rms = (time.perf_counter() - t0) * 1e3 / steps
    m.close()
    fps = train_flops_per_sample(widths)
    tflops = fps * B / (ms / 1e3) / 1e12
    nbytes = train_bytes_per_step(widths, B, m_params=sum(
        widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1)))
    return {"workload": "batch 65536 of 4096 kernels, 32-512x4-1, bf16, Adam",
            "steps_per_s": 1e3 / ms, "samples_per_s": B / (ms / 1e3), "ms_per_step": ms,
            "flops_per_sample": fps, "tflops": tflops, "peak": PEAK_TFLOPS["bf16"],
            "roofline_frac": tflops / PEAK_TFLOPS["bf16"],
            "hbm_bytes_per_step": nbytes, "hbm_gbs": nbytes / (ms / 1e3) / 1e9,
            "hbm_frac": nbytes / (ms / 1e3) / 1e9 / PEAK_HBM_GBS,
            "rmsprop_rmse_ms_per_step": ms_rms,
            "loss_last": loss_adam}


def train_bytes_per_step(widths, batch, m_params):
    """HBM bytes one bf16 training step of this design moves (saved state
    written by the forward and read back, transposed gradients written and
    read, split-K partials, optimizer state), as a second roofline for the
    step beside its flops: the step alternates matrix-core and memory phases."""
    nf, L, W = widths[0], len(widths) - 2, widths[1]
    eb = 2
    per_row = (nf * 8                       # features in (int64)
               + nf * eb + L * W * eb        # saved x^T, h_l^T
               + (L - 1) * (W // 32) * 4     # ReLU mask words
               + 4 + 8 + 4 + 4               # pred, y, dy written and read
               + W * eb + 4                  # seed: h_{L-1}^T and dy in
               + L * W * eb                  # g_l^T out
               + (L - 1) * (W // 32) * 4     # masks in
               + L * W * eb + nf * eb + (L - 1) * W * eb)  # weight gradients: g^T, x^T, h^T in
    ld = -(-batch // 256) * 256

    def splits(na, nb, cus=256):  # the library's split rule on a 256-CU device
        tiles, s = -(-na // 128) * -(-nb // 128), 1
        while tiles * s < 2 * cus and s < 64 and 2 * s * 512 <= ld:
            s *= 2
        return s
    partials = 2 * 4 * (splits(W, nf) * W * nf + (L - 1) * splits(W, W) * W * W)  # written, read back
    optimizer = m_params * 4 * 7                               # grad, master, m, v in; master, m, v out
    return int(per_row * batch + partials + optimizer)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--also", default=None,
                    help="comma-separated extra precisions timed on the same inputs ('' for none; "
                         "default: the other two of fp32, bf16 and fp8 that the workload's "
                         "network has, i.e. bf16 for the 256-wide network, fp32 for the "
                         "512-wide one, bf16 and fp32 for the 1024-wide one)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--train-steps", type=int, default=20,
                    help="timed training steps (batch 65536, bf16 32-512x4-1); 0 to skip")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--refine-k", type=int, default=None,
                    help="also time bf16/fp8 ranking refined by an fp32 model on each kernel's "
                         "top-k candidates (advisor_rank_refined; default 8 for bf16, 16 for "
                         "fp8); 0 to skip")
    ap.add_argument("--no-transfers", dest="transfers", action="store_false",
                    help="skip the leg that hands the descriptors over in pinned host memory")
    ap.add_argument("--no-stages", dest="stages", action="store_false",
                    help="skip timing advisor_featurize and advisor_rank_preds alone")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates the "
                         "HBM byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X here "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    # tuning results stay inside this run unless a cache file is named
    os.environ.setdefault("ADVISOR_TUNE_CACHE", "")
    import torch
    import paper_2301_03636_amd as adv

    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=d)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "launches": 3}), flush=True)
        return
    cfg = args.config
    prec = args.precision or DEFAULT_PRECISION[cfg]
    kd, vd, off, params, widths = make_inputs(cfg)
    nv, nk = vd.shape[0], off.size - 1

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(d)
    kdd, vdd, offd = T(kd), T(vd), T(off)
    # Z-score statistics from a seeded calibration sample, fitted on the GPU
    cal = T(workload.sample_rows(nv, 65536, workload.seeds(cfg)["desc"] + 7))
    feat_cal, inv_cal = adv.advisor_featurize(kdd, vdd[cal])
    feat_cal = feat_cal[inv_cal == 0].contiguous()
    mu_d, sd_d = adv.advisor_zscore_fit(feat_cal)
    mu, sd = mu_d.cpu().numpy(), sd_d.cpu().numpy()

    results = {}
    best_by_prec = {}
    also = args.also if args.also is not None else DEFAULT_ALSO[cfg]
    precs = [prec] + [p for p in also.split(",") if p and p != prec]
    for p in precs:
        m = adv.Model(widths, p)
        m.set_params(params, mu, sd)
        if p == "fp8":
            m.calibrate_fp8(feat_cal)
        # tile shape chosen by the library's autotuner on this workload
        shape, shape_ms = adv.advisor_autotune(m.handle, kdd, vdd, offd, reps=3)
        best = torch.empty(nk, dtype=torch.int64, device=d)
        ms, kern_ms, launches, pct = time_rank(adv, torch, m, kdd, vdd, offd, best,
                                               args.steps if p == prec else max(5, args.steps // 2),
                                               args.warmup)
        best_by_prec[p] = best.cpu().numpy()
        fl = sum(layer_flops(widths))
        results[p] = dict(ms_per_step=ms, kernel_ms=kern_ms, launches=launches,
                          value=nv / (ms / 1e3), replay_ms=pct,
                          tflops=fl * nv / (kern_ms / 1e3) / 1e12,
                          tile_shape=shape, tune_ms=[round(t, 4) for t in shape_ms[:4]],
                          mfma_peak_measured=adv.advisor_mfma_peak(p, iters=100000))
        if p == prec and args.transfers:
            results[p]["with_transfers"] = time_with_transfers(
                adv, torch, m, kd, vd, off, kdd, vdd, offd, best, max(5, args.steps // 2),
                args.warmup)
        # the prediction flow's top-10 list per kernel (fused pass + top-N), eager calls
        tidx = torch.empty((nk, 10), dtype=torch.int64, device=d)
        tval = torch.empty((nk, 10), dtype=torch.float32, device=d)
        nsteps = args.steps if p == prec else max(5, args.steps // 2)
        for _ in range(args.warmup):
            m.rank_topn(kdd, vdd, offd, 10, idx_out=tidx, val_out=tval)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            m.rank_topn(kdd, vdd, offd, 10, idx_out=tidx, val_out=tval)
        torch.cuda.synchronize()
        tms = (time.perf_counter() - t0) * 1e3 / nsteps
        results[p]["top10"] = dict(ms_per_step=tms, value=nv / (tms / 1e3),
                                   head_equals_argmin=bool(torch.equal(tidx[:, 0], best)))
        del tidx, tval
        rk = refine_k_for(p, args.refine_k)
        if p != "fp32" and rk > 0:
            # the same ranking with each kernel's top-k re-ranked in fp32 (eager calls)
            hi = adv.Model(widths, "fp32")
            hi.set_params(params, mu, sd)
            bref = torch.empty(nk, dtype=torch.int64, device=d)
            nsteps = args.steps if p == prec else max(5, args.steps // 2)
            for _ in range(args.warmup):
                m.rank_refined(hi, kdd, vdd, offd, top_k=rk, best_out=bref)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nsteps):
                m.rank_refined(hi, kdd, vdd, offd, top_k=rk, best_out=bref)
            torch.cuda.synchronize()
            rms = (time.perf_counter() - t0) * 1e3 / nsteps
            best_by_prec[p + "_refined"] = bref.cpu().numpy()
            results[p]["refined"] = dict(top_k=rk, ms_per_step=rms, value=nv / (rms / 1e3))
            hi.close()
            if p == "fp8":
                # the cheaper second stage: the fp8 model's top-k re-ranked in bf16
                mid = adv.Model(widths, "bf16")
                mid.set_params(params, mu, sd)
                for _ in range(args.warmup):
                    m.rank_refined(mid, kdd, vdd, offd, top_k=rk, best_out=bref)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(nsteps):
                    m.rank_refined(mid, kdd, vdd, offd, top_k=rk, best_out=bref)
                torch.cuda.synchronize()
                rms = (time.perf_counter() - t0) * 1e3 / nsteps
                best_by_prec["fp8_refined_bf16"] = bref.cpu().numpy()
                results[p]["refined_bf16"] = dict(top_k=rk, ms_per_step=rms, value=nv / (rms / 1e3))
                mid.close()
        m.close()
    del feat_cal, inv_cal

    main_r = results[prec]
    peak = roofline_peak(widths, prec)
    traffic = stored_traffic(cfg, prec)
    out = {
        "metric": "variants ranked/sec (featurize+MLP+argmin), BF16/FP8 vs FP32 at argmin agreement",
        "value": main_r["value"],
        "unit": "variants/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[prec],
        "data": "synthetic (seeded descriptors and He-init weights)",
        "config": {"workload": WORKLOAD_NAME[cfg], "n_kernels": nk, "n_variants": nv,
                   "widths": list(widths), "precision": prec},
        "roofline": {"bound": "mfma", "achieved": main_r["tflops"], "peak": round(peak, 1),
                     "unit": "TFLOP/s", "frac": main_r["tflops"] / peak,
                     "traffic": traffic,
                     "kernel": "mlp_tiles_kernel (fused featurize+MLP+argmin)",
                     "kernel_ms": main_r["kernel_ms"],
                     "flops_per_variant": sum(layer_flops(widths)),
                     "replay_ms": main_r["replay_ms"],
                     "mfma_peak_measured": main_r["mfma_peak_measured"]},
    }
    # variants/s per replay: p10 of the rate is the p90 of the duration
    out["value_p10_p50_p90"] = [nv / (main_r["replay_ms"][q] / 1e3) for q in ("p90", "p50", "p10")]
    if "with_transfers" in main_r:
        out["with_transfers"] = main_r["with_transfers"]
    if args.stages:
        out["stages"] = stage_kernels(adv, torch, kdd, vdd, offd, max(5, args.steps // 2))
    agree_t = {}
    if not args.no_cpu_baseline:
        cb, agree, per_variant = cpu_baseline_leg(kd, vd, off, widths, params, mu, sd,
                                                  args.cpu_seconds, best_by_prec)
        agree_t, tinfo = trained_agreement(adv, torch, T, kd, vd, off, widths, list(results),
                                           per_variant, args.cpu_seconds / 2, args.refine_k)
        cb["argmin_agreement_trained_network"] = dict(agree_t, **tinfo)
        out["cpu_baseline"] = cb
    else:
        agree = {}
    out["precisions"] = {
        p: {"value": r["value"], "ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
            "tflops": r["tflops"], "roofline_frac": r["tflops"] / roofline_peak(widths, p),
            "tile_shape": r["tile_shape"], "autotune_ms": r["tune_ms"],
            "replay_ms": r["replay_ms"], "mfma_peak_measured": r["mfma_peak_measured"],
            "top10": r.get("top10"),
            "argmin_agreement_vs_oracle_sample": agree.get(p),
            "argmin_agreement_trained_network": agree_t.get(p),
            "refined_by_fp32": None if "refined" not in r else dict(
                r["refined"], argmin_agreement_vs_oracle_sample=agree.get(p + "_refined"),
                argmin_agreement_trained_network=agree_t.get(p + "_refined")),
            "refined_by_bf16": None if "refined_bf16" not in r else dict(
                r["refined_bf16"], argmin_agreement_vs_oracle_sample=agree.get(p + "_refined_bf16"),
                argmin_agreement_trained_network=agree_t.get(p + "_refined_bf16"))}
        for p, r in results.items()}
    if args.train_steps > 0:
        out["train"] = train_leg(adv, torch, d, args.train_steps, args.warmup)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
