"""Pins of the oracle's gradient norm and of the synthetic runtime model's
target and regret, against values worked by hand and closed forms.

The norm is the float64 2-norm of the gradient that the training step
reports (the gradient-norm reduction the training step carries beside the
loss); a sum of squares without the root, an L1 norm or a dropped sign would
fail the Pythagorean vectors below. The runtime model stands in for the
measured runtimes of section 5.2 (section 3's training mode needs them); the
regret is the gain measure of the trained network against picks without it.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import cost

from test_oracle_features import WORKED_KD, WORKED_VD


@pytest.mark.parametrize("vec, norm", [
    ([3.0, 4.0], 5.0),                 # sum of squares 25, L1 7, max 4
    ([-3.0, 4.0, 12.0], 13.0),         # 9 + 16 + 144 = 169, a negative entry
    ([1.0, -2.0, 2.0], 3.0),
    ([2.0, 3.0, 6.0], 7.0),
    ([0.0, 0.0, -7.5], 7.5),           # one non-zero entry: its magnitude
    ([], 0.0),
    ([0.5] * 16, 2.0),                 # c * sqrt(n) with c = 1/2, n = 16
    ([1.0] * 1024, 32.0),              # sqrt(1024)
])
def test_l2norm_exact_values(vec, norm):
    # every value above is exact in float64 (squares, sums and roots of
    # small integers and powers of two)
    assert oracle.l2norm(np.array(vec, dtype=np.float64)) == norm


def test_l2norm_scaled_unit_vector():
    # a unit vector (entries 1/sqrt(n), signs alternating) scaled by 2.5:
    # norm 2.5 up to n roundings of the squares and the sum
    n = 4096
    v = np.full(n, 1.0 / math.sqrt(n))
    v[1::2] *= -1.0
    assert abs(oracle.l2norm(2.5 * v) - 2.5) <= 1e-12
    # homogeneity |a| ||g|| and invariance under permutation and sign flips
    rng = np.random.default_rng(91)
    g = rng.standard_normal(1000)
    base = oracle.l2norm(g)
    assert abs(oracle.l2norm(-3.0 * g) - 3.0 * base) <= 1e-12 * base
    assert abs(oracle.l2norm(rng.permutation(g) * np.sign(rng.standard_normal(1000))) - base) \
        <= 1e-12 * base


# A compute-bound variant worked by hand: one loop of 7,000,000 iterations,
# one 1-byte array of class alloc mapped alloc (nothing moves), 10 flops per
# iteration, collapse 1, 1024 teams x 128 threads. Then Pc = 7e6 parallel
# iterations, TH = 131072 = 2^17 threads, busy = 2^17, so u_c = u_m = 1;
# flops = 7e7 -> 7e7 / 7e12 = 10 us; bytes = 7e6 -> 7e6 / 9e11 = 7.8 us
# (below the compute term); no transfer; plus the 5 us launch floor:
# t = 15 us exactly, target ln 15.
COMPUTE_KD = [1, 7000000, 1, 1, 1, 1, 1, 0, 0, 0, 0, 10, 0, 0, 0, 0]
COMPUTE_VD = [0, 1, 1024, 128, 0, 0, 0, 0]


def _feat(kd, vd):
    f, inv = oracle.featurize(np.array([kd]), np.array([vd]))
    assert inv.tolist() == [0]
    return f


def test_runtime_compute_bound_by_hand():
    t = cost.runtime_s(_feat(COMPUTE_KD, COMPUTE_VD))[0]
    assert abs(t - 15e-6) <= 1e-18


def test_runtime_partial_occupancy_by_hand():
    # the same kernel with 8 teams x 1024 threads: busy = 8192 = 2^13, so the
    # compute rate drops to P * 2^13 / 2^17 = P / 16 and the memory rate to
    # B * 2^13 / 2^15 = B / 4: compute 10 us * 16 = 160 us, memory
    # 7e6 / 2.25e11 = 31.1 us; t = 160 + 5 = 165 us
    vd = list(COMPUTE_VD)
    vd[2], vd[3] = 8, 1024
    t = cost.runtime_s(_feat(COMPUTE_KD, vd))[0]
    assert abs(t - 165e-6) <= 1e-17


def test_target_worked_values():
    # no noise: the target is ln(runtime in microseconds)
    f = _feat(COMPUTE_KD, COMPUTE_VD)
    assert abs(cost.target(f, np.zeros(1))[0] - math.log(15.0)) <= 1e-14
    assert abs(cost.target(f, np.zeros(1))[0] - 2.70805020110221) <= 1e-12
    # the worked memory/transfer-bound variant: 46.683 ms -> ln 46683 = 10.75113
    fw = _feat(WORKED_KD, WORKED_VD)
    assert abs(cost.target(fw, np.zeros(1))[0] - 10.75113) <= 5e-6
    # noise enters as the factor exp(0.1 z): z = +1 adds 0.1 to the log, z = -2
    # subtracts 0.2 (sigma 0.1 of section 3's stand-in measurements)
    z = np.array([1.0, -2.0, 0.5])
    y = cost.target(np.repeat(f, 3, axis=0), z)
    assert np.allclose(y, math.log(15.0) + np.array([0.1, -0.2, 0.05]), rtol=0, atol=1e-13)


def test_regret_worked_by_hand():
    # kernel 0: runtimes 2, 1, 4, pick the first -> 2/1 - 1 = 1
    # kernel 1: runtimes 3, 3, pick the second (a tie with the best) -> 0
    # kernel 2: runtimes 5, 10, 2.5, 20, pick the last -> 20/2.5 - 1 = 7
    # kernel 3: one variant, picked -> 0
    t = np.array([2.0, 1.0, 4.0, 3.0, 3.0, 5.0, 10.0, 2.5, 20.0, 0.25])
    off = np.array([0, 3, 5, 9, 10])
    pick = np.array([0, 4, 8, 9])
    assert cost.regret(t, off, pick).tolist() == [1.0, 0.0, 7.0, 0.0]
    # picking each kernel's fastest variant has no regret
    assert cost.regret(t, off, np.array([1, 3, 7, 9])).tolist() == [0.0, 0.0, 0.0, 0.0]


def test_regret_two_variant_kernel_by_hand():
    # The worked kernel with two variants: the worked one (maps to, from,
    # tofrom, alloc) and one mapping array 0 tofrom instead of to. Both share
    # the memory term 11 * 2^27 B / (9e11 * 4096 / 2^15 B/s) = 13.1235 ms.
    # Variant A moves 2S to and 2S back (S = 2^27 B): 2^29 B / 16 GB/s =
    # 33.5544 ms, t_A = 46.6829 ms. Variant B moves 2S to and 3S back:
    # 5 * 2^27 B / 16 GB/s = 41.9430 ms, t_B = 55.0716 ms.
    vb = list(WORKED_VD)
    vb[4] = 3
    f = np.vstack([_feat(WORKED_KD, WORKED_VD), _feat(WORKED_KD, vb)])
    t = cost.runtime_s(f)
    mem = 11 * 2.0 ** 27 / (9e11 * 4096 / 2.0 ** 15)
    assert abs(mem - 0.01312351118) < 1e-11
    assert abs(t[0] - (mem + 2.0 ** 29 / 1.6e10 + 5e-6)) <= 1e-15
    assert abs(t[1] - (mem + 5 * 2.0 ** 27 / 1.6e10 + 5e-6)) <= 1e-15
    off = np.array([0, 2])
    # picking B costs t_B / t_A - 1 = 55.07155 / 46.68294 - 1 = 0.179693
    r = cost.regret(t, off, np.array([1]))[0]
    assert abs(r - 0.179693) <= 1e-6
    assert cost.regret(t, off, np.array([0]))[0] == 0.0
