"""Pins of the oracle's generated-variant descriptors: section 4.1.3's
variants (parallel-for position x, teams collapse d, parallel-for collapse c,
schedule, data option) lowered to cost-model descriptor rows and featurized.

Checked against feature vectors worked by hand for a split directive and for
a nest with a serial loop between the two directives, an exact
Python-integer evaluation of the definitions on every variant the generator
makes for random nests, the invariants that tie the features together, the
data options against the data analysis (section 4.1.2: analysed maps move
between one half and all of what mapping everything both ways moves), and
the combined placement against the benchmark descriptors."""
import numpy as np
import pytest

import oracle
import workload

# the worked kernel of the feature pins: 3-deep nest 16 x 256 x 4096, four
# 8-byte arrays (array 1 strided), 8 flops per iteration, classes
# (to, from, tofrom, alloc)
KD = [3, 16, 256, 4096, 1, 4, 8, 0, 1, 0, 0, 8, 1, 2, 3, 0]


def _cf(x, d, c, s):
    return c + 8 * x + 64 * d + 512 * s


def test_split_directive_worked_example():
    """teams distribute collapse(1) at loop 0, parallel for collapse(2) at
    loop 1, dynamic schedule, 64 teams x 256 threads. By hand: the teams share
    Pt = 16 iterations, each team's threads Pf = 256 * 4096 = 1048576, so the
    parallel space is 2^24 = I and nothing runs serially (R = 1); 3 loops are
    collapsed; busy = min(64, 16) * min(256, 2^20) = 4096 threads; waves =
    ceil(16 / 64) * ceil(2^20 / 256) = 4096; idle slots 4096 * 16384 - 2^24
    = 50331648. The data features are those of the combined worked variant."""
    vd = [0, _cf(1, 1, 2, 1), 64, 256, 1, 2, 3, 0]
    f, inv = oracle.featurize(np.array([KD]), np.array([vd]))
    assert inv.tolist() == [0]
    expect = [3, 16, 256, 4096, 1, 16777216, 3, 16777216, 1, 64, 256, 16384, 4096, 4096, 4096,
              50331648, 4, 8, 134217728, 1, 1, 1, 1, 268435456, 268435456, 536870912, 1,
              536870912, 1476395008, 134217728, 8, 134217728]
    assert f[0].tolist() == expect


def test_serial_loop_between_the_directives():
    """A 4-deep nest 8 x 16 x 32 x 64: teams over loop 0 (8 iterations),
    loop 1 run by each team, parallel for over loop 2 (32 iterations), loop 3
    serial inside. By hand: Pc = 8 * 32 = 256, R = 16 * 64 = 1024, two
    collapsed loops; 4 teams x 64 threads: busy = 4 * 32 = 128, waves =
    ceil(8 / 4) * ceil(32 / 64) = 2, waves * R = 2048, idle = 2 * 256 - 256."""
    kd = [4, 8, 16, 32, 64, 1, 8, 0, 0, 0, 0, 1, 3, 0, 0, 0]
    vd = [0, _cf(2, 1, 1, 0), 4, 64, 3, 0, 0, 0]
    f, inv = oracle.featurize(np.array([kd]), np.array([vd]))
    assert inv.tolist() == [0]
    assert f[0, 5:16].tolist() == [262144, 2, 256, 1024, 4, 64, 256, 128, 2, 2048, 256]


def _bigint(kd, vd):
    """Python-integer evaluation of the feature definitions for any parallel
    structure (None for an invalid variant)."""
    k = [int(v) for v in kd[int(vd[0])]]
    D, N, A, E, s, fpi, req = k[0], k[1:5], k[5], k[6], k[7:11], k[11], k[12:16]
    cf, T, H, m = int(vd[1]), int(vd[2]), int(vd[3]), [int(v) for v in vd[4:8]]
    allowed = {0: {0, 1, 2, 3}, 1: {1, 3}, 2: {2, 3}, 3: {3}}
    if not (0 <= cf < 1536) or T < 1 or H < 1:
        return None
    c, x, d, sch = cf % 8, (cf // 8) % 8, (cf // 64) % 8, cf // 512
    if x == 0 and not (d == 0 and 1 <= c <= D):
        return None
    if x >= 1 and not (x < D and 1 <= d <= x and 1 <= c <= D - x):
        return None
    for a in range(A):
        if m[a] not in allowed[req[a]]:
            return None
    prod = lambda lo, hi: int(np.prod([N[i] for i in range(lo, hi)], dtype=object)) if hi > lo else 1  # noqa: E731
    I = prod(0, 4)
    TH = T * H
    if x == 0:
        Pc, R = prod(0, c), prod(c, 4)
        busy, waves, npar = min(TH, Pc), -(-Pc // TH), c
    else:
        Pt, Pf = prod(0, d), prod(x, x + c)
        Pc, R = Pt * Pf, prod(d, x) * prod(x + c, 4)
        busy, waves, npar = min(T, Pt) * min(H, Pf), (-(-Pt // T)) * (-(-Pf // H)), d + c
    S = E * I
    cnt = [sum(1 for a in range(A) if m[a] == q) for q in range(4)]
    ns = sum(s[:A])
    h2d, d2h = S * (cnt[1] + cnt[3]), S * (cnt[2] + cnt[3])
    return [D, N[0], N[1], N[2], N[3], I, npar, Pc, R, T, H, TH, busy, waves, waves * R,
            waves * TH - Pc, A, E, S, cnt[1], cnt[2], cnt[3], cnt[0], h2d, d2h, h2d + d2h, ns,
            S * A, S * (A - ns) + (64 // E) * S * ns, fpi * I, fpi, S * cnt[0]]


@pytest.mark.parametrize("depth", [1, 2, 3, 4, "mixed"])
def test_generated_variants_bigint(depth):
    kd, _, _ = workload.make_descriptors(30, 1, 2, seed=61 + (depth if depth != "mixed" else 9),
                                         depth=depth)
    off, gen = oracle.enumerate_variants(kd[:, 0])
    assert off[-1] == int(np.sum(kd[:, 0] ** 3 + 5 * kd[:, 0]))
    for teams, threads in ((64, 256), (1, 1), (4096, 1024)):
        vd = oracle.lower_variants(kd, gen, teams, threads)
        f, inv = oracle.featurize(kd, vd)
        assert not inv.any()   # every generated variant is a valid descriptor
        for i in range(vd.shape[0]):
            assert f[i].tolist() == _bigint(kd, vd[i])
        # invariants: parallel part times serial part is the whole nest; the
        # rounds of work cover the parallel space; threads that get work fit
        # the launch and the work
        assert np.all(f[:, 7] * f[:, 8] == f[:, 5])
        assert np.all(f[:, 13] * f[:, 11] >= f[:, 7])
        assert np.all(f[:, 12] <= np.minimum(f[:, 11], f[:, 7]))
        assert np.all((f[:, 6] >= 1) & (f[:, 6] <= f[:, 0]))


def test_structure_rules():
    """Invalid structures: teams collapse at the combined placement, none or
    deeper than x at a split one, a parallel-for collapse past the nest, the
    directive past the last loop, an unknown schedule, stray high bits."""
    ok = [(0, 0, 1, 0), (0, 0, 3, 2), (1, 1, 2, 1), (2, 2, 1, 0), (2, 1, 1, 2)]
    bad = [(0, 1, 1, 0), (1, 0, 1, 0), (1, 2, 1, 0), (1, 1, 3, 0), (3, 1, 1, 0), (0, 0, 4, 0),
           (0, 0, 0, 0), (1, 1, 2, 3)]
    vds = [[0, _cf(*t), 64, 256, 1, 2, 3, 0] for t in ok + bad] + \
          [[0, -586, 64, 256, 1, 2, 3, 0], [0, 1536 + 1, 64, 256, 1, 2, 3, 0]]
    _, inv = oracle.featurize(np.array([KD]), np.array(vds))
    assert inv.tolist() == [0] * len(ok) + [1] * (len(bad) + 2)


def test_lowering_maps_and_data_options():
    """Data option 0 maps each array with its analysed class, option 1 maps
    every array tofrom: the second moves between one and two times the
    bytes of the first when no array is alloc (exactly two when every array
    is read-only or write-only, as for Wilson Dslash in section 5.1), and
    variants that differ only in their schedule have identical features."""
    kd, _, _ = workload.make_descriptors(200, 1, 2, seed=71, depth="mixed")
    off, gen = oracle.enumerate_variants(kd[:, 0])
    vd = oracle.lower_variants(kd, gen, 128, 256)
    k = gen[:, 0]
    A = kd[k, 5]
    arr = np.arange(4)[None, :] < A[:, None]
    assert np.array_equal(vd[gen[:, 5] == 0, 4:8], np.where(arr, kd[k, 12:16], 0)[gen[:, 5] == 0])
    assert np.all(vd[gen[:, 5] == 1, 4:8][arr[gen[:, 5] == 1]] == 3)
    assert np.all(vd[:, 2] == 128) and np.all(vd[:, 3] == 256)
    assert np.array_equal(vd[:, 1], gen[:, 3] + 8 * gen[:, 1] + 64 * gen[:, 2] + 512 * gen[:, 4])
    f, inv = oracle.featurize(kd, vd)
    assert not inv.any()
    # rows come in (schedule, data) blocks of six per placement
    f6 = f.reshape(-1, 3, 2, 32)
    assert np.all(f6[:, 0] == f6[:, 1]) and np.all(f6[:, 0] == f6[:, 2])
    an, nv = f6[:, 0, 0, 25], f6[:, 0, 1, 25]
    no_alloc = np.all(kd[gen[::6, 0], 12:16][:, :4] != 0, axis=1) & (kd[gen[::6, 0], 5] == 4)
    r = nv[no_alloc] / an[no_alloc]
    assert no_alloc.any() and r.min() >= 1.0 and r.max() <= 2.0
    pure = no_alloc & np.all(kd[gen[::6, 0], 12:16] != 3, axis=1)
    assert pure.any() and np.all(nv[pure] == 2 * an[pure])


def test_combined_placement_is_the_benchmark_descriptor():
    """A generated variant at x = 0 with collapse c is the descriptor the
    benchmark workloads use (collapse c of the combined directive): same row
    with the static schedule, same features with any schedule."""
    kd, vd_b, _ = workload.make_descriptors(50, 20, 21, seed=81)
    off, gen = oracle.enumerate_variants(kd[:, 0])
    comb = gen[gen[:, 1] == 0]
    lo = oracle.lower_variants(kd, comb, 256, 128)
    static = comb[:, 4] == 0
    b = np.zeros((comb.shape[0], 8), dtype=np.int64)
    b[:, 0], b[:, 1], b[:, 2], b[:, 3] = comb[:, 0], comb[:, 3], 256, 128
    b[:, 4:8] = lo[:, 4:8]
    assert np.array_equal(lo[static], b[static])
    fa, _ = oracle.featurize(kd, lo)
    fb, _ = oracle.featurize(kd, b)
    assert np.array_equal(fa, fb)
