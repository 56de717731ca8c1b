"""Pins of the oracle's random numbers (theta_ij of the random force, Eq. random).

Philox4x32-10 is checked against the generator's published known-answer
values; the Box-Muller normals against the moments of N(0, 1); the pair
symmetry theta_ij = theta_ji (needed for momentum conservation) directly.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    out = orc.philox4x32_10(ctr, key)
    assert [int(x) for x in out] == expect


def test_uniform23_exact_in_single_precision(orc):
    for x in [0, 1, 511, 512, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0x12345678]:
        u = orc.uniform23(x)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
    assert orc.uniform23(0) == 2.0 ** -24
    assert orc.uniform23(0xFFFFFFFF) == 1.0 - 2.0 ** -24


def test_theta_symmetric_in_pair(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        i, j = (int(x) for x in rng.integers(0, 1 << 20, size=2))
        step, box = int(rng.integers(0, 1 << 31)), int(rng.integers(0, 4096))
        seed = int(rng.integers(0, 1 << 62))
        assert orc.theta(seed, i, j, step, box) == orc.theta(seed, j, i, step, box)


def test_theta_moments_standard_normal(orc):
    n = 120_000
    seed = 0x4C484D4D0000
    vals = np.array([orc.theta(seed, k, k + 1 + (k % 7), k // 13, k % 5) for k in range(n)])
    se = 1.0 / math.sqrt(n)
    assert abs(vals.mean()) < 5 * se
    assert abs(vals.var() - 1.0) < 5 * math.sqrt(2.0) * se
    kurt = np.mean(vals ** 4) / vals.var() ** 2
    assert abs(kurt - 3.0) < 5 * math.sqrt(24.0) * se
    # tail mass beyond 2 sigma of a unit normal: 0.0455
    tail = np.mean(np.abs(vals) > 2.0)
    assert abs(tail - 0.0455) < 5 * math.sqrt(0.0455 * 0.9545 / n)


def test_theta_changes_with_every_counter_word(orc):
    seed = 77
    base = orc.theta(seed, 3, 9, 100, 2)
    assert orc.theta(seed, 4, 9, 100, 2) != base
    assert orc.theta(seed, 3, 10, 100, 2) != base
    assert orc.theta(seed, 3, 9, 101, 2) != base
    assert orc.theta(seed, 3, 9, 100, 3) != base
    assert orc.theta(seed + 1, 3, 9, 100, 2) != base
    assert orc.theta(seed + (1 << 32), 3, 9, 100, 2) != base
