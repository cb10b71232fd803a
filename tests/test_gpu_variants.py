"""Variant generation (section 4.1.3) on the GPU against the oracle's
enumeration, bit for bit: the paper's kernels, random loop counts including
values outside 1..4, every schedule mask, enough kernels for the offsets'
prefix sum to span many blocks and several passes of its block-sum scan,
and offsets that do not match the counts (rows stay in bounds, the extra
rows read -1)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
from gpu_util import host, say, to_dev

pytestmark = pytest.mark.gpu


def _gpu(n_loops, mask):
    off, rows = adv.advisor_enumerate_variants(to_dev(np.asarray(n_loops, np.int64)), mask)
    return host(off), host(rows)


def test_paper_kernels():
    # the kernels of the code-generation table, by loop count
    nl = [1, 1, 1, 1, 1, 2, 2, 2, 1, 2, 1, 2, 1, 1, 1, 1, 1, 1, 1, 4, 4]
    off, rows = _gpu(nl, 7)
    ro, rr = oracle.enumerate_variants(nl, 7)
    assert np.array_equal(off, ro) and np.array_equal(rows, rr)
    counts = np.diff(off)
    assert counts.tolist() == [n ** 3 + 5 * n for n in nl]


@pytest.mark.parametrize("mask", [1, 2, 3, 4, 5, 6, 7])
def test_random_loop_counts_every_mask(mask):
    rng = np.random.default_rng(500 + mask)
    nl = rng.integers(-2, 7, size=5000)
    nl[:3] = [0, 1 << 40, -(1 << 40)]
    say("variants mask=%d n_k=%d" % (mask, nl.size))
    off, rows = _gpu(nl, mask)
    ro, rr = oracle.enumerate_variants(nl, mask)
    assert np.array_equal(off, ro)
    assert np.array_equal(rows, rr)


def test_many_kernels_spanning_scan_blocks():
    """300,000 kernels: 293 scan blocks of 1024 kernels, so the block-sum scan
    takes two passes of 256. Offsets are checked in full, rows on a seeded
    sample of whole kernels and on the last kernels."""
    rng = np.random.default_rng(510)
    nk = 300000
    nl = rng.integers(0, 6, size=nk)
    table_off, _ = oracle.enumerate_variants(np.arange(0, 6), 7)
    per_n = np.diff(table_off)
    want_off = np.concatenate([[0], np.cumsum(per_n[nl])]).astype(np.int64)
    say("variants n_k=%d n_v=%d" % (nk, want_off[-1]))
    off, rows = _gpu(nl, 7)
    assert np.array_equal(off, want_off)
    ks = np.concatenate([rng.choice(nk, 2000, replace=False), np.arange(nk - 5, nk)])
    for k in ks:
        _, rr = oracle.enumerate_variants([nl[k]], 7)
        got = rows[off[k]:off[k + 1]]
        assert got.shape[0] == rr.shape[0]
        if rr.shape[0]:
            assert np.all(got[:, 0] == k) and np.array_equal(got[:, 1:], rr[:, 1:])


def test_empty_and_mismatched_offsets():
    e = adv.advisor_count_variants(torch.empty(0, dtype=torch.int64, device="cuda"))
    assert host(e).tolist() == [0]
    nl = np.array([4, 2, 3], np.int64)
    d_nl = to_dev(nl)
    off7 = adv.advisor_count_variants(d_nl, 7)
    _, rows = adv.advisor_enumerate_variants(d_nl, 1, offsets=off7)
    rows, o = host(rows), host(off7)
    _, rr = oracle.enumerate_variants(nl, 1)
    ro, _ = oracle.enumerate_variants(nl, 1)
    for k in range(3):
        cnt = ro[k + 1] - ro[k]
        seg = rows[o[k]:o[k + 1]]
        assert np.array_equal(seg[:cnt, 1:], rr[ro[k]:ro[k + 1], 1:])
        assert np.all(seg[:cnt, 0] == k) and np.all(seg[cnt:] == -1)
