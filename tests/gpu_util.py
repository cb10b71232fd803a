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
