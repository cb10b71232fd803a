"""Helpers shared by the GPU tests: device placement and tolerances."""
import sys

import numpy as np
import torch


def dev():
    assert torch.cuda.is_available(), "GPU tests need an MI355X; none is visible"
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(p, r):
    """|p - r| / max(|r|, 1): relative error on ln(us), absolute near 0."""
    p = np.asarray(p, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    return np.abs(p - r) / np.maximum(np.abs(r), 1.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def segment_argmin(pred, offsets):
    """Per segment, the lowest index holding the smallest non-NaN value, or
    -1 when the segment is empty or all NaN. Plain numpy (an fmin reduction
    per segment), independent of the library and of the oracle: it checks
    that the library's argmin is exact on the library's own predictions."""
    pred = np.asarray(pred, dtype=np.float64)
    off = np.asarray(offsets, dtype=np.int64)
    nk = off.size - 1
    best = np.full(nk, -1, dtype=np.int64)
    counts = np.diff(off)
    nz = np.nonzero(counts)[0]
    if nz.size == 0:
        return best
    assert pred.size == off[-1]
    segmin = np.full(nk, np.nan)
    segmin[nz] = np.fmin.reduceat(pred, off[nz])
    seg = np.repeat(np.arange(nk), counts)
    idx = np.nonzero(pred == segmin[seg])[0]
    s = seg[idx]
    first = np.ones(idx.size, dtype=bool)
    first[1:] = s[1:] != s[:-1]
    best[s[first]] = idx[first]
    return best


def elementwise_grad_err(g, g_ref, widths):
    """Worst element-by-element error of a gradient, per weight matrix and
    bias vector: max |g - r| / max(|r|, s), where s is the RMS of the
    reference entries of that matrix or vector (the floor keeps entries that
    cancel to nearly 0 from demanding a relative accuracy no summation order
    gives them). Returns the worst ratio over all parts."""
    g = np.asarray(g, np.float64)
    worst, off = 0.0, 0
    for i in range(len(widths) - 1):
        for k in (widths[i + 1] * widths[i], widths[i + 1]):
            r = g_ref[off:off + k]
            s = float(np.sqrt(np.mean(r * r)))
            if s > 0.0:
                worst = max(worst, float(np.max(np.abs(g[off:off + k] - r) / np.maximum(np.abs(r), s))))
            else:
                assert np.all(g[off:off + k] == 0.0)
            off += k
    return worst
