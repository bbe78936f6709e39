"""Pins of the oracle's windowed 2-opt (2-opt with a small probability,
Section 4; moves limited to edges within W tour positions, Section 5).

Every check below is computed here without the oracle's gain formula:
* a hand-worked square with one crossing (gains, chosen move, result);
* points in convex position: a 2-optimal tour over all edge pairs is the
  hull order, of length the polygon's perimeter;
* local optimality against brute force: every 2-opt neighbour within the
  window, built by reversing a segment and measured in full, is no shorter;
* the length changes by exactly the reported gain, the tour stays a
  permutation, and rounds are memoryless (stopping after r rounds and
  restarting gives the same tour);
* two defects far apart are both repaired in one round;
* tours take part with probability p."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances


def _d(xy, a, b):
    """nint Euclidean distance, exact for |coordinates| <= 2^26 (no half-integer ties)."""
    dx = xy[a, 0].astype(np.int64) - xy[b, 0]
    dy = xy[a, 1].astype(np.int64) - xy[b, 1]
    return np.rint(np.sqrt((dx * dx + dy * dy).astype(np.float64))).astype(np.int64)


def _length(xy, t):
    t = np.asarray(t)
    return int(_d(xy, t, np.roll(t, -1)).sum())


def _neighbours_no_shorter(xy, t, window):
    """Every 2-opt neighbour whose removed edges start at most `window` positions apart
    (cyclically): reverse t[i+1..j] and measure the whole tour."""
    n = len(t)
    L = _length(xy, t)
    W = min(window, n - 2)
    for i in range(n):
        for o in range(2, W + 1):
            pos = [(i + 1 + q) % n for q in range(o)]
            u = np.array(t)
            u[pos] = u[pos[::-1]]
            if _length(xy, u) < L:
                return False, (i, o)
    return True, None


def _is_perm(t, n):
    return np.array_equal(np.sort(t), np.arange(n))


def test_square_with_one_crossing_by_hand():
    # tour 0-2-1-3 on the square (0,0) (10,0) (10,10) (0,10): edges 14+10+14+10 = 48.
    # Position 0 (t0=0, t1=2, t2=1, t3=3): d(0,1)+d(2,3)-d(0,2)-d(1,3) = 10+10-14-14 = -8;
    # position 2 the same move from the other side (-8); positions 1 and 3 give 0.
    # Both spans overlap; the tie goes to position 0; reversing t1..t2 gives 0-1-2-3 (40).
    xy = np.array([[0, 0], [10, 0], [10, 10], [0, 10]], np.int32)
    g, o = orc.two_opt_best(xy, [0, 2, 1, 3], 500)
    np.testing.assert_array_equal(g, [-8, 0, -8, 0])
    np.testing.assert_array_equal(o, [2, 0, 2, 0])
    t, st = orc.two_opt(xy, [0, 2, 1, 3], 500)
    np.testing.assert_array_equal(t, [0, 1, 2, 3])
    assert st == dict(rounds=1, moves=1, gain=-8, converged=True)


def _polygon(n, R=10**6, seed=0):
    ang = 2 * np.pi * np.arange(n) / n
    return np.stack([np.rint(R * np.cos(ang)), np.rint(R * np.sin(ang))], 1).astype(np.int32)


def _hull_order(t):
    n = len(t)
    r = np.roll(t, -int(np.argmin(t)))
    return np.array_equal(r, np.arange(n)) or np.array_equal(np.r_[r[:1], r[1:][::-1]],
                                                             np.arange(n))


@pytest.mark.parametrize("n", [8, 40, 97])
def test_convex_position_reaches_the_hull_order(n):
    xy = _polygon(n)
    rng = np.random.default_rng(n)
    for _ in range(3):
        t0 = rng.permutation(n).astype(np.int32)
        t, st = orc.two_opt(xy, t0, 500)
        assert st["converged"]
        assert _hull_order(t), t
        assert _length(xy, t) == _length(xy, np.arange(n))
        assert _length(xy, t) - _length(xy, t0) == st["gain"]


@pytest.mark.parametrize("n,window", [(5, 500), (7, 500), (9, 3), (12, 4), (60, 7), (60, 500)])
def test_result_is_locally_optimal_by_brute_force(n, window):
    rng = np.random.default_rng(100 + n + window)
    xy = rng.integers(0, 1000, (n, 2)).astype(np.int32)
    xy = np.unique(xy, axis=0)
    n = len(xy)
    for rep in range(3):
        t0 = rng.permutation(n).astype(np.int32)
        t, st = orc.two_opt(xy, t0, window)
        assert st["converged"] and _is_perm(t, n)
        ok, mv = _neighbours_no_shorter(xy, t, window)
        assert ok, (rep, mv)
        assert _length(xy, t) - _length(xy, t0) == st["gain"]
        assert st["moves"] >= st["rounds"] and (st["gain"] < 0) == (st["moves"] > 0)


def test_gain_accounting_and_memoryless_rounds():
    xy = instances.uniform_coords(2000, 11, hi=1_000_000)
    n = len(xy)
    t0 = np.random.default_rng(5).permutation(n).astype(np.int32)
    full, st = orc.two_opt(xy, t0, 50)
    assert st["converged"] and _is_perm(full, n)
    assert _length(xy, full) - _length(xy, t0) == st["gain"]
    part, s1 = orc.two_opt(xy, t0, 50, max_rounds=3)
    assert s1["rounds"] == 3 and not s1["converged"]
    assert _length(xy, part) - _length(xy, t0) == s1["gain"]
    rest, s2 = orc.two_opt(xy, part, 50)
    np.testing.assert_array_equal(rest, full)
    assert s1["rounds"] + s2["rounds"] == st["rounds"]
    assert s1["moves"] + s2["moves"] == st["moves"]
    # the first round applies the best move of all, and more besides
    g, o = orc.two_opt_best(xy, t0, 50)
    _, r1 = orc.two_opt(xy, t0, 50, max_rounds=1)
    assert r1["gain"] <= g.min() and r1["moves"] > 1


def test_two_far_defects_repaired_in_one_round():
    n = 60
    xy = _polygon(n)
    t0 = np.arange(n, dtype=np.int32)
    t0[[10, 11]] = t0[[11, 10]]
    t0[[40, 41]] = t0[[41, 40]]
    t, st = orc.two_opt(xy, t0, 500, max_rounds=1)
    np.testing.assert_array_equal(t, np.arange(n))
    assert st["rounds"] == 1 and st["moves"] == 2


def test_degenerate_sizes_and_windows():
    xy = np.array([[0, 0], [5, 0], [0, 5]], np.int32)
    t, st = orc.two_opt(xy, [0, 2, 1], 500)
    np.testing.assert_array_equal(t, [0, 2, 1])
    assert st == dict(rounds=0, moves=0, gain=0, converged=True)
    xy = _polygon(30)
    t0 = np.random.default_rng(1).permutation(30).astype(np.int32)
    t, st = orc.two_opt(xy, t0, 1)        # a window below 2 allows no move
    np.testing.assert_array_equal(t, t0)
    assert st["moves"] == 0


def test_participation_probability():
    for p in (0.0, 1.0):
        sel = [orc.two_opt_selected(7, 3, a, p) for a in range(500)]
        assert all(sel) == (p == 1.0) and any(sel) == (p == 1.0)
    p = 0.05
    sel = np.array([orc.two_opt_selected(7, it, a, p) for it in range(20) for a in range(1000)])
    sd = np.sqrt(p * (1 - p) / len(sel))
    assert abs(sel.mean() - p) < 5 * sd
    # independent of PartialACO's partial draw (word 1 of the same block)
    part = np.array([orc.partial_plan(7, it, a, 1000, 0.5, 10)[1] for it in range(20)
                     for a in range(1000)])
    both = (sel & part).mean()
    assert abs(both - p * 0.5) < 5 * np.sqrt(p * 0.5 * (1 - p * 0.5) / len(sel))
