"""Synthetic runtime model (test infrastructure).

The paper trains its network on runtimes measured by compiling and running
every variant on the target machine (sections 3 and 5.2). Those measurements
are not available here, so a closed-form roofline-style runtime stands in for
them; it is the thing the network learns, not part of the method:

  t = max(flops / (P * u_c), bytes / (B * u_m)) + transfer / LINK + 5 us

with u_c = min(busy, 2^17) / 2^17 and u_m = min(busy, 2^15) / 2^15 the shares
of the machine the launch keeps busy, P = 7e12 flop/s, B = 9e11 B/s and
LINK = 1.6e10 B/s; observed runtimes carry log-normal noise exp(0.1 z), and
the regression target is ln(runtime in microseconds).
"""
from __future__ import annotations

import numpy as np

P_FLOPS = 7.0e12
B_BYTES = 9.0e11
LINK = 1.6e10
LAUNCH = 5e-6
NOISE_SIGMA = 0.1


def runtime_s(feat: np.ndarray) -> np.ndarray:
    """Noise-free runtime in seconds from oracle features (float64)."""
    f = np.asarray(feat)
    busy = f[:, 12].astype(np.float64)
    u_c = np.minimum(busy, 2.0 ** 17) / 2.0 ** 17
    u_m = np.minimum(busy, 2.0 ** 15) / 2.0 ** 15
    flops = f[:, 29].astype(np.float64)
    bytes_ = f[:, 28].astype(np.float64)
    xfer = f[:, 25].astype(np.float64)
    return np.maximum(flops / (P_FLOPS * u_c), bytes_ / (B_BYTES * u_m)) + xfer / LINK + LAUNCH


def target(feat: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Noisy log-runtime target ln(t * exp(0.1 z) * 1e6)."""
    t = runtime_s(feat) * np.exp(NOISE_SIGMA * np.asarray(z, dtype=np.float64))
    return np.log(t * 1e6)


def regret(t_true: np.ndarray, offsets: np.ndarray, pick: np.ndarray) -> np.ndarray:
    """Per kernel, t(pick) / min_i t(i) - 1 under the noise-free runtime."""
    out = np.zeros(offsets.size - 1)
    for k in range(offsets.size - 1):
        seg = t_true[offsets[k]:offsets[k + 1]]
        out[k] = t_true[pick[k]] / seg.min() - 1.0
    return out
