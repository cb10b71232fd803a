"""The oracle's data analysis (section 4.1.2) against what the paper fixes:
each of the five class definitions on the access pattern it describes, the
enter/exit-data split, the bound that mapping everything to and from the GPU
moves between one and two times the analysed bytes (which every pair of
figure plot:data obeys, Wilson Dslash at exactly two), and agreement with the
featurizer's transfer features for a variant that maps each array with its
analysed class."""
import os

import numpy as np

import oracle
import workload

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BEFORE, READ, WRITE, AFTER, LOCAL = 1, 2, 4, 8, 16
ALLOC, TO, FROM, TOFROM, PRIVATE, NONE = range(6)


def test_each_definition():
    # alloc: assigned within for the first time, no transfer to the GPU
    assert oracle.map_class(WRITE) == ALLOC
    assert oracle.map_class(WRITE | READ) == ALLOC
    # to: assigned before, only read within
    assert oracle.map_class(BEFORE | READ) == TO
    assert oracle.map_class(BEFORE | READ | AFTER) == TO
    # from: updated within, accessed after, nothing to send in
    assert oracle.map_class(WRITE | AFTER) == FROM
    assert oracle.map_class(WRITE | READ | AFTER) == FROM
    # tofrom: assigned before, updated within, accessed after
    assert oracle.map_class(BEFORE | WRITE | AFTER) == TOFROM
    assert oracle.map_class(BEFORE | READ | WRITE | AFTER) == TOFROM
    # private: defined and used only within the kernel
    for b in range(16):
        assert oracle.map_class(LOCAL | b) == PRIVATE
    # not used by the kernel at all
    assert oracle.map_class(BEFORE | AFTER) == NONE and oracle.map_class(0) == NONE


def test_directions_follow_the_classes():
    """alloc, to and tofrom enter with the enter-data directive; only to and
    tofrom carry bytes in, from and tofrom carry bytes out."""
    acc = np.array([WRITE, BEFORE | READ, WRITE | AFTER, BEFORE | WRITE | AFTER, LOCAL | READ,
                    BEFORE], dtype=np.uint8)
    nb = np.array([1, 10, 100, 1000, 10000, 100000], dtype=np.int64)
    cls, e, x, nv = oracle.classify(acc, nb, [0, 6])
    assert cls.tolist() == [ALLOC, TO, FROM, TOFROM, PRIVATE, NONE]
    assert e.tolist() == [1010] and x.tolist() == [1100] and nv.tolist() == [2 * 1111]


def test_naive_over_analysed_between_one_and_two():
    """Mapping everything to and from the GPU moves each byte twice; the
    analysis moves every to/from/tofrom byte at least once, so without
    alloc variables the ratio lies in [1, 2]: 1 when every variable is
    tofrom, 2 when every variable is pure to or pure from."""
    rng = np.random.default_rng(30)
    mapped = [b for b in range(16) if oracle.map_class(b) in (TO, FROM, TOFROM)]
    for _ in range(200):
        n = int(rng.integers(1, 9))
        acc = rng.choice(mapped, n).astype(np.uint8)
        nb = rng.integers(1, 1 << 30, n)
        _, e, x, nv = oracle.classify(acc, nb, [0, n])
        r = nv[0] / (e[0] + x[0])
        assert 1.0 <= r <= 2.0
    acc = np.full(4, BEFORE | READ | WRITE | AFTER, np.uint8)
    _, e, x, nv = oracle.classify(acc, np.full(4, 7, np.int64), [0, 4])
    assert nv[0] == e[0] + x[0]
    acc = np.array([BEFORE | READ] * 3 + [WRITE | AFTER], np.uint8)
    _, e, x, nv = oracle.classify(acc, np.full(4, 3 << 27, np.int64), [0, 4])
    assert nv[0] == 2 * (e[0] + x[0])


def test_figure_pairs_obey_the_bound():
    rows = []
    with open(os.path.join(GOLD, "data_transfer_gb.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, b, a = line.split()
                rows.append((name, float(b), float(a)))
    assert len(rows) == 12
    for name, b, a in rows:
        assert 1.0 - 1e-9 <= b / a <= 2.0 + 0.02, name  # printed to two decimals
    wil = [r for r in rows if r[0] == "wilson_dslash"][0]
    assert wil[1] / wil[2] == 2.0


def test_transfer_features_agree_with_analysis():
    """A variant mapping every array with its analysed class: the
    featurizer's h2d and d2h features (f23, f24) equal the analysis's
    enter and exit bytes when each array spans the whole loop nest."""
    kd, vd, off = workload.make_descriptors(50, 1, 4, 40)
    rng = np.random.default_rng(41)
    mapped = [b for b in range(16) if oracle.map_class(b) in (ALLOC, TO, FROM, TOFROM)]
    for k in range(kd.shape[0]):
        A = int(kd[k, 5])
        acc = rng.choice(mapped, A).astype(np.uint8)
        I = int(np.prod(kd[k, 1:5]))
        S = int(kd[k, 6]) * I
        cls, e, x, _ = oracle.classify(acc, np.full(A, S, np.int64), [0, A])
        kk = kd[k].copy()
        kk[12:12 + A] = cls
        v = np.array([[0, 1, 64, 64, 0, 0, 0, 0]], dtype=np.int64)
        v[0, 4:4 + A] = cls
        f, inv = oracle.featurize(kk[None, :], v)
        assert inv[0] == 0
        assert f[0, 23] == e[0] and f[0, 24] == x[0]
