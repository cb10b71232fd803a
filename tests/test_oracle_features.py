"""Pins of the oracle's feature extraction, Z-score and synthetic runtime.

The oracle is checked against things other than itself: a feature vector
worked by hand from the feature definitions, exact Python-integer
recomputation, algebraic invariants that tie features together, the data
volumes the paper reports before and after its data analysis, and library
statistics for the Z-score.
"""
import numpy as np
import pytest

import oracle
import workload
from oracle import cost

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

# kernel: 3-deep nest 16 x 256 x 4096, four 8-byte arrays, array 1 strided,
# 8 flops per iteration, data classes (to, from, tofrom, alloc)
WORKED_KD = [3, 16, 256, 4096, 1, 4, 8, 0, 1, 0, 0, 8, 1, 2, 3, 0]
# variant: collapse 2, 64 teams x 256 threads, maps (to, from, tofrom, alloc)
WORKED_VD = [0, 2, 64, 256, 1, 2, 3, 0]
# worked by hand from the feature definitions: I = 16*256*4096 = 2^24,
# Pc = 16*256 = 4096, R = 4096, TH = 16384, busy = 4096, waves = 1,
# S = 8 * 2^24 = 2^27, h2d = d2h = 2S, strided bytes = 3S + 8*1*S = 11S ...
WORKED_F = [3, 16, 256, 4096, 1, 16777216, 2, 4096, 4096, 64, 256, 16384, 4096, 1, 4096,
            12288, 4, 8, 134217728, 1, 1, 1, 1, 268435456, 268435456, 536870912, 1,
            536870912, 1476395008, 134217728, 8, 134217728]


def test_worked_example():
    f, inv = oracle.featurize(np.array([WORKED_KD]), np.array([WORKED_VD]))
    assert inv.tolist() == [0]
    assert f[0].tolist() == WORKED_F


def test_worked_example_runtime():
    # roofline-style runtime of the worked variant: memory term
    # 11 * 2^27 B / (9e11 B/s / 8) = 13.12 ms, transfer 2^29 B / 16 GB/s
    # = 33.55 ms, plus 5 us -> 46.683 ms, i.e. ln(46683 us) = 10.75113
    f, _ = oracle.featurize(np.array([WORKED_KD]), np.array([WORKED_VD]))
    t = cost.runtime_s(f)[0]
    assert abs(t - 0.0466829) < 5e-8
    assert abs(np.log(t * 1e6) - 10.75113) < 5e-6


def _features_bigint(kd, vd, n_k):
    """Python-integer evaluation of the feature definitions (no wrap-around)."""
    kid = int(vd[0])
    if not (0 <= kid < n_k):
        return None
    k = [int(v) for v in kd[kid]]
    D, N, A, E = k[0], k[1:5], k[5], k[6]
    s, fpi, req = k[7:11], k[11], k[12:16]
    c, T, H, m = int(vd[1]), int(vd[2]), int(vd[3]), [int(v) for v in vd[4:8]]
    allowed = {0: {0, 1, 2, 3}, 1: {1, 3}, 2: {2, 3}, 3: {3}}
    if not (1 <= D <= 4) or any(n < 1 for n in N) or any(N[i] != 1 for i in range(D, 4)):
        return None
    if not (0 <= A <= 4) or not (1 <= E <= 64) or fpi < 0:
        return None
    if not (1 <= c <= D) or T < 1 or H < 1:
        return None
    for a in range(A):
        if s[a] not in (0, 1) or req[a] not in allowed or m[a] not in allowed[req[a]]:
            return None
    I = N[0] * N[1] * N[2] * N[3]
    Pc = 1
    for i in range(c):
        Pc *= N[i]
    R = I // Pc
    TH = T * H
    busy = min(TH, Pc)
    waves = -(-Pc // TH)
    S = E * I
    cnt = [sum(1 for a in range(A) if m[a] == q) for q in range(4)]
    ns = sum(s[:A])
    h2d = S * (cnt[1] + cnt[3])
    d2h = S * (cnt[2] + cnt[3])
    line = 64 // E
    return [D, N[0], N[1], N[2], N[3], I, c, Pc, R, T, H, TH, busy, waves, waves * R,
            waves * TH - Pc, A, E, S, cnt[1], cnt[2], cnt[3], cnt[0], h2d, d2h, h2d + d2h, ns,
            S * A, S * (A - ns) + line * S * ns, fpi * I, fpi, S * cnt[0]]


@pytest.mark.parametrize("depth", [1, 2, 3, 4, "mixed"])
def test_bigint_recompute(depth):
    kd, vd, off = workload.make_descriptors(40, 1, 24, seed=11 + (depth if depth != "mixed" else 9),
                                            depth=depth, invalid_frac=0.15)
    f, inv = oracle.featurize(kd, vd)
    for i in range(vd.shape[0]):
        ref = _features_bigint(kd, vd[i], kd.shape[0])
        if ref is None:
            assert inv[i] == 1 and not f[i].any()
        else:
            assert inv[i] == 0
            assert max(ref) < 2 ** 63
            assert f[i].tolist() == ref


def test_invariants():
    kd, vd, off = workload.make_descriptors(300, 16, 200, seed=5, depth="mixed")
    f, inv = oracle.featurize(kd, vd)
    f = f[inv == 0].astype(object)  # python ints: no overflow in the checks
    assert f.shape[0] > 10000
    # transfer volume is the sum of both directions
    assert all(f[:, 25] == f[:, 23] + f[:, 24])
    # every array falls in exactly one map class
    assert all(f[:, 19] + f[:, 20] + f[:, 21] + f[:, 22] == f[:, 16])
    # collapsed part times serial part is the whole iteration space
    assert all(f[:, 7] * f[:, 8] == f[:, 5])
    # waves is the ceiling of collapsed iterations over threads
    assert all(f[:, 13] * f[:, 11] >= f[:, 7])
    assert all((f[:, 13] - 1) * f[:, 11] < f[:, 7])
    # busy threads are bounded by both the launch and the exposed work
    assert all(f[:, 12] <= np.minimum(f[:, 11], f[:, 7]))
    # idle slots of the last wave are non-negative and below one launch
    assert all((f[:, 15] >= 0) & (f[:, 15] < f[:, 11]))
    # strided walks only add bytes: unit-stride volume <= penalized volume
    assert all(f[:, 27] <= f[:, 28])
    # product of the trip counts
    assert all(f[:, 1] * f[:, 2] * f[:, 3] * f[:, 4] == f[:, 5])


def test_all_alloc_moves_nothing():
    kd = np.array([[2, 64, 64, 1, 1, 3, 4, 0, 1, 1, 0, 2, 0, 0, 0, 0]])
    vd = np.array([[0, 1, 128, 64, 0, 0, 0, 0], [0, 2, 128, 64, 3, 0, 1, 0]])
    f, inv = oracle.featurize(kd, vd)
    assert inv.tolist() == [0, 0]
    assert f[0, 23] == f[0, 24] == f[0, 25] == 0
    assert f[0, 31] == 3 * f[0, 18]
    assert f[1, 23] == 2 * f[1, 18] and f[1, 24] == f[1, 18]


def test_bytes_rule_against_paper_volumes():
    """Section 5.1 reports transfer volumes before the data analysis (every
    array copied both ways) and after it: the reduction is between 1x and 2x
    for all twelve applications, and exactly 2x (1.5 GB -> 0.75 GB) for the
    Wilson Dslash operator, whose arrays are each read-only or write-only.
    The map-clause byte rule must reproduce that bracket."""
    rng = np.random.default_rng(3)
    kd, vd, off = workload.make_descriptors(200, 4, 4, seed=21)
    kd[:, 12:16] = rng.integers(1, 4, size=(200, 4))           # no alloc class
    for i in range(vd.shape[0]):                               # analysed maps: minimal
        vd[i, 4:8] = kd[vd[i, 0], 12:16]
    f_an, inv = oracle.featurize(kd, vd)
    assert not inv.any()
    vd_naive = vd.copy()
    vd_naive[:, 4:8] = 3                                       # naive: tofrom everything
    f_nv, _ = oracle.featurize(kd, vd_naive)
    ratio = f_nv[:, 25] / f_an[:, 25]
    assert ratio.min() >= 1.0 and ratio.max() <= 2.0
    pure = (kd[vd[:, 0], 12:16] != 3).all(axis=1)
    assert pure.any() and np.all(ratio[pure] == 2.0)
    # 1.5 GB before, 0.75 GB after for the Dslash shape (four read-only or
    # write-only arrays): the ratio is exactly the paper's 2
    assert 1.5 / 0.75 == 2.0


@pytest.mark.parametrize("field,value", [
    ("c", 0), ("c", 4), ("T", 0), ("H", -1), ("kid", -1), ("kid", 1), ("N", 0), ("D", 0),
    ("D", 5), ("E", 0), ("A", 5), ("map", 0), ("s", 2), ("fpi", -1), ("Nunused", 2),
])
def test_invalid_rules(field, value):
    kd = np.array([WORKED_KD])
    vd = np.array([WORKED_VD])
    if field == "c":
        vd[0, 1] = value
    elif field == "T":
        vd[0, 2] = value
    elif field == "H":
        vd[0, 3] = value
    elif field == "kid":
        vd[0, 0] = value
    elif field == "N":
        kd[0, 2] = value
    elif field == "D":
        kd[0, 0] = value
    elif field == "E":
        kd[0, 6] = value
    elif field == "A":
        kd[0, 5] = value
    elif field == "map":
        vd[0, 4] = value          # array 0 needs host->device data: alloc drops it
    elif field == "s":
        kd[0, 7] = value
    elif field == "fpi":
        kd[0, 11] = value
    elif field == "Nunused":
        kd[0, 4] = value          # loop 3 does not exist at depth 3
    f, inv = oracle.featurize(kd, vd)
    assert inv.tolist() == [1]
    assert not f.any()


def test_wraparound_is_defined():
    """Beyond the no-overflow domain the features are the values modulo 2^64
    (two's complement), never undefined."""
    kd = np.array([[4, 4096, 4096, 4096, 4096, 4, 64, 1, 1, 1, 1, 1024, 3, 3, 3, 3]])
    vd = np.array([[0, 4, 1, 1, 3, 3, 3, 3]])
    f, inv = oracle.featurize(kd, vd)
    assert inv.tolist() == [0]
    I = 4096 ** 4
    S = 64 * I

    def wrap(v):
        v %= 2 ** 64
        return v - 2 ** 64 if v >= 2 ** 63 else v
    assert f[0, 5] == wrap(I)
    assert f[0, 18] == wrap(S)
    assert f[0, 29] == wrap(1024 * I)


def test_zscore_matches_library_statistics():
    kd, vd, off = workload.make_descriptors(100, 16, 300, seed=8)
    f, inv = oracle.featurize(kd, vd)
    mu, sd = oracle.zscore_fit(f)
    L = np.log2(f.astype(np.float64) + 1.0)
    ref_mu = L.mean(axis=0)
    ref_sd = L.std(axis=0, ddof=0)
    const = f.min(axis=0) == f.max(axis=0)
    ref_sd[const] = 1.0
    assert const[[0, 4, 16, 17]].all() and const.sum() == 4
    assert np.allclose(mu, ref_mu, rtol=1e-12, atol=1e-12)
    assert np.allclose(sd, ref_sd, rtol=1e-10, atol=1e-12)
    x = oracle.normalize(f, mu, sd)
    # constant features (depth, arrays, element size, unused loop) map to 0
    for j in (0, 4, 16, 17):
        assert sd[j] == 1.0 and np.all(x[:, j] == 0.0)
    # the calibration sample itself is standardized
    var = ~const
    assert np.allclose(x[:, var].mean(axis=0), 0.0, atol=1e-9)
    assert np.allclose(x[:, var].std(axis=0), 1.0, atol=1e-9)


def test_synthetic_targets_span_paper_range():
    """The stand-in runtimes cover roughly the 0.04 s - 48 s span of the
    Wilson Dslash variants the paper plots, down to tens of microseconds."""
    kd, vd, off = workload.make_descriptors(400, 16, 256, seed=1004)
    f, inv = oracle.featurize(kd, vd)
    t = cost.runtime_s(f[inv == 0])
    assert t.min() >= 5e-6 and t.max() < 1e3
    assert t.min() < 1e-3 and t.max() > 10.0
    y = cost.target(f[inv == 0], workload.noise(t.size, 3004))
    assert np.all(y > np.log(5.0) - 0.5)
