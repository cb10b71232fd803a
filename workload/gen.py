"""Seeded synthetic inputs for the cost-model hot path.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic (no features, no network, no ranking). Both the HIP
path and the CPU oracle consume what it produces.

Descriptor layout (int64, row-major):

  kdesc [n_kernels, 16]: D, N0, N1, N2, N3, A, E, s0, s1, s2, s3, fpi,
                         req0, req1, req2, req3
      D       loop-nest depth (number of nested for loops, section 4.1.1)
      N_i     trip count of loop i (N_i = 1 for i >= D)
      A       number of arrays the kernel touches, E bytes per element
      s_a     1 if array a is walked with a stride of N, 0 if unit stride
      fpi     flops per innermost iteration
      req_a   data class the live-variable analysis assigns to array a
              (section 4.1.2): 0 alloc, 1 to, 2 from, 3 tofrom
  vdesc [n_variants, 8]: kernel_id, c, T, H, m0, m1, m2, m3
      c       collapse depth of the combined teams-distribute-parallel-for
      T, H    number of teams and threads per team
      m_a     map clause chosen for array a (same codes as req_a)
  offsets [n_kernels + 1]: CSR segment bounds; the variants of kernel k are
      rows offsets[k] .. offsets[k+1]-1 of vdesc.

Distributions follow the synthetic workload recipe: 3-deep nests with trip
counts log-uniform on [2^4, 2^12], four 8-byte arrays with unit or stride-N
access, flops per iteration 2^U{0..10}, a uniform data class per array,
collapse U{1..D}, teams 2^U{6..12}, threads 2^U{5..10}, and map clauses drawn
uniformly among the clauses that move at least the data the class needs.
"""
from __future__ import annotations

import numpy as np

KD_COLS = 16
VD_COLS = 8
N_FEATURES = 32

ALLOC, TO, FROM, TOFROM = 0, 1, 2, 3

# Map clauses that carry at least the data a class needs (section 4.1.2):
# an alloc array may be mapped any way, a to array needs the host->device
# copy, a from array the device->host copy, a tofrom array both.
_ALLOWED = {
    ALLOC: (ALLOC, TO, FROM, TOFROM),
    TO: (TO, TOFROM),
    FROM: (FROM, TOFROM),
    TOFROM: (TOFROM,),
}

# The five workloads: (kernels, min variants, max variants, layer widths).
WORKLOADS = {
    1: dict(n_kernels=1, count_lo=256, count_hi=256, widths=(32, 64, 64, 1)),
    2: dict(n_kernels=4096, count_lo=16, count_hi=1024, widths=(32, 256, 256, 256, 1)),
    3: dict(n_kernels=16384, count_lo=64, count_hi=1024, widths=(32, 512, 512, 512, 512, 1)),
    4: dict(n_kernels=4096, count_lo=16, count_hi=1024, widths=(32, 512, 512, 512, 512, 1),
            batch=65536),
    5: dict(n_kernels=32768, count_lo=128, count_hi=1024, widths=(32, 1024, 1024, 1024, 1024, 1)),
}


def seeds(cfg: int) -> dict:
    """Seeds of a workload: descriptors, weights and measurement noise."""
    return dict(desc=1000 + cfg, w=2000 + cfg, noise=3000 + cfg)


def make_descriptors(n_kernels: int, count_lo: int, count_hi: int, seed: int,
                     depth=3, n_arrays: int = 4, elem_bytes: int = 8,
                     invalid_frac: float = 0.0, counts=None):
    """Draw kdesc, vdesc and offsets.

    depth: an int (every kernel that deep) or "mixed" (U{1..4} per kernel).
    invalid_frac: share of variants corrupted into invalid ones (collapse
      deeper than the nest, zero teams, a map that drops needed data, or a
      kernel id out of range), to exercise the invalid-variant rules.
    counts: optional explicit per-kernel variant counts (overrides lo/hi).
    """
    rng = np.random.default_rng(seed)
    nk = int(n_kernels)
    if depth == "mixed":
        D = rng.integers(1, 5, size=nk)
    else:
        D = np.full(nk, int(depth), dtype=np.int64)
    kd = np.zeros((nk, KD_COLS), dtype=np.int64)
    kd[:, 0] = D
    u = rng.random((nk, 4))
    trips = np.clip(np.floor(2.0 ** (4.0 + 8.0 * u)), 16, 4096).astype(np.int64)
    loop = np.arange(4)[None, :]
    kd[:, 1:5] = np.where(loop < D[:, None], trips, 1)
    kd[:, 5] = n_arrays
    kd[:, 6] = elem_bytes
    arr = np.arange(4)[None, :] < n_arrays
    kd[:, 7:11] = np.where(arr, rng.integers(0, 2, size=(nk, 4)), 0)
    kd[:, 11] = 2 ** rng.integers(0, 11, size=nk)
    kd[:, 12:16] = np.where(arr, rng.integers(0, 4, size=(nk, 4)), 0)

    if counts is None:
        counts = rng.integers(count_lo, count_hi + 1, size=nk)
    counts = np.asarray(counts, dtype=np.int64)
    offsets = np.zeros(nk + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    nv = int(offsets[-1])
    if nv >= 2 ** 32:
        raise ValueError("variant count must stay below 2^32")

    kid = np.repeat(np.arange(nk, dtype=np.int64), counts)
    vd = np.zeros((nv, VD_COLS), dtype=np.int64)
    vd[:, 0] = kid
    Dv = D[kid]
    vd[:, 1] = 1 + np.floor(rng.random(nv) * Dv).astype(np.int64)
    vd[:, 2] = 2 ** rng.integers(6, 13, size=nv)
    vd[:, 3] = 2 ** rng.integers(5, 11, size=nv)
    # map clause per array: uniform over the clauses allowed for its class
    table = np.full((4, 4), -1, dtype=np.int64)
    sizes = np.zeros(4, dtype=np.int64)
    for r, allowed in _ALLOWED.items():
        table[r, :len(allowed)] = allowed
        sizes[r] = len(allowed)
    req = kd[kid, 12:16]
    pick = np.floor(rng.random((nv, 4)) * sizes[req]).astype(np.int64)
    m = table[req, pick]
    vd[:, 4:8] = np.where(np.arange(4)[None, :] < n_arrays, m, 0)

    if invalid_frac > 0.0:
        bad = np.nonzero(rng.random(nv) < invalid_frac)[0]
        how = rng.integers(0, 4, size=bad.size)
        for sel, kind in ((bad[how == 0], 0), (bad[how == 1], 1),
                          (bad[how == 2], 2), (bad[how == 3], 3)):
            if sel.size == 0:
                continue
            if kind == 0:      # collapse deeper than the loop nest
                vd[sel, 1] = D[vd[sel, 0]] + 1
            elif kind == 1:    # zero teams
                vd[sel, 2] = 0
            elif kind == 2:    # array 0 mapped alloc although it needs data
                k = vd[sel, 0]
                needs = kd[k, 12] != ALLOC
                vd[sel[needs], 4] = ALLOC
                vd[sel[~needs], 3] = 0
            else:              # kernel id out of range
                vd[sel, 0] = nk + 7
    return kd, vd, offsets


def param_count(widths) -> int:
    return sum(widths[i + 1] * widths[i] + widths[i + 1] for i in range(len(widths) - 1))


def he_init(widths, seed: int, bias_scale: float = 0.0) -> np.ndarray:
    """He-normal weights N(0, 2/fan_in) drawn in float64 and rounded to the
    float32 master copy; biases zero unless bias_scale > 0 (then N(0, s^2),
    used by tests to exercise the bias path).

    Layout: for each layer l, W_l as [out, in] row-major, then b_l [out].
    """
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(widths) - 1):
        fan_in, fan_out = widths[i], widths[i + 1]
        w = rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)
        if bias_scale > 0.0:
            b = rng.standard_normal(fan_out) * bias_scale
        else:
            b = np.zeros(fan_out)
        parts.append(w.ravel())
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)


def glorot_init(widths, seed: int) -> np.ndarray:
    """Glorot (Xavier) uniform weights U(-a, a), a = sqrt(6 / (fan_in +
    fan_out)), drawn in float64 and rounded to the float32 master copy, and
    zero biases: the initialization section 5.3 names. Same layout as
    he_init."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(widths) - 1):
        fan_in, fan_out = widths[i], widths[i + 1]
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def sample_rows(n_rows: int, n_sample: int, seed: int) -> np.ndarray:
    """Sorted seeded sample of row indices without replacement."""
    rng = np.random.default_rng(seed)
    n_sample = min(int(n_sample), int(n_rows))
    return np.sort(rng.choice(int(n_rows), size=n_sample, replace=False))


def sample_kernels(offsets: np.ndarray, n_sample: int, seed: int):
    """Seeded subset of whole kernels: returns (kernel ids, row indices,
    the subset's own CSR offsets)."""
    nk = offsets.size - 1
    ks = sample_rows(nk, n_sample, seed)
    counts = offsets[ks + 1] - offsets[ks]
    rows = np.concatenate([np.arange(offsets[k], offsets[k + 1]) for k in ks]) \
        if ks.size else np.zeros(0, dtype=np.int64)
    sub_off = np.zeros(ks.size + 1, dtype=np.int64)
    np.cumsum(counts, out=sub_off[1:])
    return ks, rows.astype(np.int64), sub_off


def noise(n: int, seed: int) -> np.ndarray:
    """Standard-normal draws for the log-normal measurement noise."""
    return np.random.default_rng(seed).standard_normal(int(n))


def make_config(cfg: int, **overrides):
    """Descriptors and float32 master weights of one of the five workloads."""
    c = dict(WORKLOADS[cfg])
    c.update(overrides)
    s = seeds(cfg)
    kd, vd, off = make_descriptors(c["n_kernels"], c["count_lo"], c["count_hi"], s["desc"])
    params = he_init(c["widths"], s["w"])
    return dict(kdesc=kd, vdesc=vd, offsets=off, params=params, widths=tuple(c["widths"]),
                seeds=s)


def calibration_rows(cfg: int, n_rows: int, n_sample: int = 65536) -> np.ndarray:
    """Rows of a workload's seeded calibration sample (the variants the
    Z-score statistics and the fp8 activation scales are fitted on)."""
    return sample_rows(n_rows, n_sample, seeds(cfg)["desc"] + 7)


def agreement_kernels(cfg: int, offsets: np.ndarray, n_sample: int):
    """The seeded sample of whole kernels on which argmin agreement with the
    oracle is measured (same return values as sample_kernels)."""
    return sample_kernels(offsets, n_sample, 7000 + cfg)


def inputs_digest(*arrays) -> str:
    """SHA-256 of the bytes of the given arrays (dtype and shape included):
    identifies the exact inputs a stored expected value was computed on."""
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()
