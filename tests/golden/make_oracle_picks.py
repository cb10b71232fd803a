"""Writes the float64 oracle's per-kernel picks on seeded samples of whole
kernels of the two low-precision benchmark workloads, so that GPU tests and
the benchmark can measure argmin agreement on thousands of kernels without
re-running minutes of float64 CPU work each time.

Calls only the oracle and the seeded input generator. For each workload:
the descriptors, offsets and He-initialized float32 weights of
workload.make_config, the Z-score statistics fitted by the oracle on the
workload's calibration sample, and the oracle's prediction flow (featurize,
Z-score, network, per-kernel argmin, section 3) on the kernels of
workload.agreement_kernels. Output, tests/golden/oracle_picks_cfg<c>.npz:
  kernels  int64 [n]  kernel ids of the sample (ascending)
  best     int64 [n]  the oracle's pick, a global variant index (-1: none)
  best_pred float64 [n]  its predicted ln(runtime in us)
  margin   float64 [n]  gap between the best and second-best prediction of
                        the kernel (ln us; inf with fewer than two)
  digest   the SHA-256 of the inputs (descriptors, offsets, weights)
Usage: python tests/golden/make_oracle_picks.py [cfg ...] (default 3 5).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload  # noqa: E402

# kernels per sample: about 4.6M variants of the 512-wide network and 2.4M
# of the 1024-wide one (similar float64 work, ~1.5e13 flops each)
SAMPLE = {3: 8192, 5: 4096}
CHUNK = 256


def path_for(cfg: int) -> str:
    return os.path.join(HERE, "oracle_picks_cfg%d.npz" % cfg)


def make(cfg: int, threads: int) -> None:
    t0 = time.time()
    c = workload.make_config(cfg)
    kd, vd, off, params, widths = c["kdesc"], c["vdesc"], c["offsets"], c["params"], c["widths"]
    digest = workload.inputs_digest(kd, vd, off, params)
    cal = workload.calibration_rows(cfg, vd.shape[0])
    f, inv = oracle.featurize(kd, vd[cal])
    mu, sd = oracle.zscore_fit(f[inv == 0])
    ks, rows, sub_off = workload.agreement_kernels(cfg, off, SAMPLE[cfg])
    best = np.full(ks.size, -1, dtype=np.int64)
    best_pred = np.full(ks.size, np.nan)
    margin = np.full(ks.size, np.inf)
    p64 = params.astype(np.float64)
    print("cfg %d: %d kernels, %d variants, inputs %s (%.1f s)"
          % (cfg, ks.size, rows.size, digest[:16], time.time() - t0), flush=True)
    for c0 in range(0, ks.size, CHUNK):
        c1 = min(ks.size, c0 + CHUNK)
        r0, r1 = sub_off[c0], sub_off[c1]
        vsub = vd[rows[r0:r1]].copy()
        local_off = sub_off[c0:c1 + 1] - r0
        vsub[:, 0] = np.repeat(np.arange(c1 - c0), np.diff(local_off))
        b, pred = oracle.rank(kd[ks[c0:c1]], vsub, local_off, widths, p64, mu, sd,
                              n_threads=threads, want_pred=True)
        for j in range(c1 - c0):
            if b[j] < 0:
                continue
            seg = pred[local_off[j]:local_off[j + 1]]
            best[c0 + j] = rows[r0 + b[j]]
            best_pred[c0 + j] = pred[b[j]]
            fin = np.sort(seg[np.isfinite(seg)])
            if fin.size >= 2:
                margin[c0 + j] = fin[1] - fin[0]
        print("cfg %d: %d / %d kernels (%.0f s)" % (cfg, c1, ks.size, time.time() - t0),
              flush=True)
    np.savez_compressed(path_for(cfg), kernels=ks.astype(np.int64), best=best,
                        best_pred=best_pred, margin=margin,
                        digest=np.frombuffer(digest.encode(), dtype=np.uint8))


def load(cfg: int) -> dict:
    """The stored picks (no pickled objects are read)."""
    with np.load(path_for(cfg), allow_pickle=False) as z:
        out = {k: z[k] for k in z.files}
    out["digest"] = bytes(out["digest"]).decode()
    return out


if __name__ == "__main__":
    cfgs = [int(a) for a in sys.argv[1:]] or [3, 5]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    for cfg in cfgs:
        make(cfg, threads)
