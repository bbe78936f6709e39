"""Pins for the oracle's integer distance d = nint(sqrt(dx^2 + dy^2)) (Section 2).

Reference: Python's exact integer square root.  nint(sqrt(s)) = r + 1 exactly
when 4s > 4r^2 + 4r + 1 - 1, with r = isqrt(s) (sqrt(s) is never r + 1/2)."""
import math
import random

import numpy as np


def ref_nint(s: int) -> int:
    r = math.isqrt(s)
    return r + 1 if 4 * s > 4 * r * r + 4 * r else r


def test_hand_values(orc):
    xy = np.array([[0, 0], [3, 4], [1, 1], [1, 2], [2, 3], [-5, -12]], np.int32)
    assert orc.dist(xy, 0, 1) == 5          # 3-4-5 triangle
    assert orc.dist(xy, 0, 2) == 1          # sqrt 2 = 1.414
    assert orc.dist(xy, 0, 3) == 2          # sqrt 5 = 2.236
    assert orc.dist(xy, 0, 4) == 4          # sqrt 13 = 3.606
    assert orc.dist(xy, 0, 5) == 13         # 5-12-13
    assert orc.dist(xy, 1, 5) == orc.dist(xy, 5, 1)


def test_exhaustive_small(orc):
    lib = orc.lib()
    for s in range(0, 300_000):
        assert lib.oracle_nint_sqrt(s) == ref_nint(s), s


def test_half_integer_neighbourhood(orc):
    rng = random.Random(5)
    lib = orc.lib()
    for _ in range(20_000):
        r = rng.randrange(1, 3_000_000_000)
        for s in (r * r + r - 1, r * r + r, r * r + r + 1, r * r, r * r - 1):
            if 0 <= s < 2**63:
                assert lib.oracle_nint_sqrt(s) == ref_nint(s), s


def test_random_large(orc):
    rng = random.Random(6)
    lib = orc.lib()
    for _ in range(50_000):
        s = rng.randrange(0, 2**62)
        assert lib.oracle_nint_sqrt(s) == ref_nint(s), s


def test_tour_length_matches_numpy(orc):
    rng = np.random.default_rng(3)
    xy = rng.integers(-1000, 1000, size=(50, 2)).astype(np.int32)
    tour = rng.permutation(50).astype(np.int32)
    ref = sum(ref_nint(int(((xy[tour[t]] - xy[tour[(t + 1) % 50]]).astype(np.int64) ** 2).sum()))
              for t in range(50))
    assert orc.tour_length(xy, tour) == ref
