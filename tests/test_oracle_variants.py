"""The oracle's variant generation (section 4.1.3) against what the paper
fixes: the variant counts of its two tables, the closed form n^3 + 5n, a
brute-force filter of every candidate tuple by the placement rules, and the
listing of Code lst:advisor:for_loops as one of the generated variants."""
import itertools
import os

import numpy as np

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table():
    rows = []
    with open(os.path.join(GOLD, "variants_per_kernel.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                app, kern, loops, nv = line.split()
                rows.append((app, kern, int(loops), int(nv)))
    return rows


def test_counts_match_both_tables():
    rows = _table()
    assert len(rows) == 4 + 21
    off, _ = oracle.enumerate_variants([r[2] for r in rows])
    assert np.diff(off).tolist() == [r[3] for r in rows]


def test_closed_form():
    """n placements at loop 0 plus x (n - x) at each later loop, times three
    schedules and two data options: 6 (n + sum x (n - x)) = n^3 + 5n."""
    for n in range(1, 5):
        off, _ = oracle.enumerate_variants([n])
        assert off[-1] == n ** 3 + 5 * n
        placements = n + sum(x * (n - x) for x in range(1, n))
        assert off[-1] == 6 * placements


def test_brute_force_rule_filter():
    """Every tuple (x, d, c, schedule, data) over generous ranges, kept when
    it obeys the placement rules, is generated exactly once, and nothing
    else is generated."""
    for n in range(1, 5):
        want = set()
        for x, d, c, s, t in itertools.product(range(6), range(6), range(6), range(3), range(2)):
            if x >= n or c < 1:
                continue
            if x == 0 and d == 0 and c <= n:
                want.add((x, d, c, s, t))
            if x >= 1 and 1 <= d <= x and c <= n - x:
                want.add((x, d, c, s, t))
        _, rows = oracle.enumerate_variants([n])
        got = [tuple(r) for r in rows[:, 1:].tolist()]
        assert len(got) == len(set(got)) and set(got) == want


def test_schedule_mask_and_invalid_loop_counts():
    """Compilers without dynamic or guided scheduling on the GPU (section
    5.1) leave a third of the variants: static only gives (n^3 + 5n) / 3."""
    off, rows = oracle.enumerate_variants([4, 3], sched_mask=1)
    assert np.diff(off).tolist() == [28, 14] and np.all(rows[:, 4] == 0)
    off, _ = oracle.enumerate_variants([0, -1, 5, 2, 1 << 40], sched_mask=7)
    assert np.diff(off).tolist() == [0, 0, 0, 18, 0]
    off, _ = oracle.enumerate_variants([3], sched_mask=0)
    assert off[-1] == 0


def test_listing_variant_is_generated():
    """Code lst:advisor:for_loops: four loops, teams distribute collapse(1)
    at loop 0, parallel for collapse(3) schedule(static) at loop 1."""
    _, rows = oracle.enumerate_variants([4])
    assert sum(1 for r in rows.tolist() if r[1:5] == [1, 1, 3, 0]) == 2  # both data options
