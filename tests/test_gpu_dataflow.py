"""Data analysis (section 4.1.2) on the GPU against the oracle, bit for bit:
every access pattern, kernels with no variables and with more variables than
a wave has lanes, sizes up to 2^40 bytes, and 200,000 kernels."""
import numpy as np
import pytest

import oracle
import paper_2301_03636_amd as adv
from gpu_util import host, say, to_dev

pytestmark = pytest.mark.gpu


def _case(nk, lo, hi, seed):
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, nk)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    acc = rng.integers(0, 32, off[-1]).astype(np.uint8)
    nb = rng.integers(0, 1 << 40, off[-1]).astype(np.int64)
    return acc, nb, off


@pytest.mark.parametrize("nk,lo,hi,seed", [(1, 0, 0, 1), (300, 0, 12, 2), (40, 60, 200, 3),
                                           (200000, 0, 8, 4)])
def test_classify_bit_exact(nk, lo, hi, seed):
    acc, nb, off = _case(nk, lo, hi, seed)
    say("classify n_k=%d n_vars=%d" % (nk, acc.size))
    got = [host(t) for t in adv.advisor_classify_maps(to_dev(acc), to_dev(nb), to_dev(off))]
    ref = oracle.classify(acc, nb, off)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_every_pattern_once():
    acc = np.arange(32, dtype=np.uint8)
    nb = (np.int64(1) << np.arange(32, dtype=np.int64))
    off = np.array([0, 32], dtype=np.int64)
    cls, e, x, n = (host(t) for t in adv.advisor_classify_maps(to_dev(acc), to_dev(nb), to_dev(off)))
    assert cls.tolist() == [oracle.map_class(b) for b in range(32)]
    rc, re, rx, rn = oracle.classify(acc, nb, off)
    assert e.tolist() == re.tolist() and x.tolist() == rx.tolist() and n.tolist() == rn.tolist()
