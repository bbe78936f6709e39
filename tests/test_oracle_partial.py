"""Pins of the PartialACO oracle (Section 3.1, Algorithm 1; the cap and the
probability of partial modification, Section 4).

* p = 0: every ant builds a full tour, identical to the plain construction;
* r = 1: the one free city is forced, so the tour is the local best rotated to
  start at the planned position;
* exact rational probabilities of the rebuilt part (n = 7), from the kept
  cities as the visited set;
* the plan's draws: start position uniform on [0, n), rebuilt count uniform on
  [1, M], partial share p, M clamped to [1, n-1];
* the local best is replaced only by a strictly shorter tour."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as orc
from oracle import exact
from paper_1709_03187_amd import instances


def _instance(n, k, seed):
    xy = instances.uniform_coords(n, seed, hi=10_000)
    nn, nnd = orc.knn_rows(xy, k)
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0.5, 2.0, (n, k)).astype(np.float32)
    return xy, nn, nnd, tau


def _local_bests(xy, nn, nnd, tau, m, seed):
    """Full tours of iteration 0 as the ants' local bests."""
    res = orc.construct(xy, nn, nnd, tau, 1.0, 2.0, seed, 0, np.arange(m))
    return res["tours"], res["lengths"]


def test_probability_zero_is_the_plain_construction():
    xy, nn, nnd, tau = _instance(300, 8, 1)
    lb, _ = _local_bests(xy, nn, nnd, tau, 12, 5)
    for it in (1, 2):
        full = orc.construct(xy, nn, nnd, tau, 1.0, 2.0, 5, it, np.arange(12), want_slots=True,
                             want_probs=True)
        part = orc.construct_partial(xy, nn, nnd, tau, 1.0, 2.0, 5, it, np.arange(12), lb, 0.0,
                                     30)
        np.testing.assert_array_equal(part["tours"], full["tours"])
        np.testing.assert_array_equal(part["lengths"], full["lengths"])
        np.testing.assert_array_equal(part["probs"], full["probs"])
        np.testing.assert_array_equal(part["slots"], full["slots"])


def test_one_rebuilt_city_gives_the_rotated_local_best():
    xy, nn, nnd, tau = _instance(200, 8, 2)
    lb, lbl = _local_bests(xy, nn, nnd, tau, 10, 7)
    part = orc.construct_partial(xy, nn, nnd, tau, 1.0, 2.0, 7, 3, np.arange(10), lb, 1.0, 1)
    for a in range(10):
        s, partial, r = orc.partial_plan(7, 3, a, 200, 1.0, 1)
        assert partial and r == 1
        np.testing.assert_array_equal(part["tours"][a], np.roll(lb[a], -s))
        assert part["lengths"][a] == lbl[a]


def test_rebuilt_part_has_exact_probabilities():
    n, k = 7, 6
    xy, nn, nnd, tau = _instance(n, k, 3)
    pts = [tuple(map(int, p)) for p in xy]
    lb, _ = _local_bests(xy, nn, nnd, tau, 1, 11)
    checked = 0
    for it in range(1, 120):
        ant = it % 5
        res = orc.construct_partial(xy, nn, nnd, tau, 1.0, 2.0, 11, it, [ant], lb, 1.0, 4)
        T = res["tours"][0]
        s, partial, r = orc.partial_plan(11, it, ant, n, 1.0, 4)
        keep = n - r
        assert list(T[:keep]) == [int(lb[0][(s + t) % n]) for t in range(keep)]
        assert sorted(T) == list(range(n))
        assert res["lengths"][0] == exact.tour_length(pts, list(T))
        visited = set(int(c) for c in T[:keep])
        p_exact = Fraction(1)
        for t in range(keep, n):
            dist = exact.step_distribution(int(T[t - 1]), visited, pts, nn.tolist(), nnd.tolist(),
                                           tau)
            p_exact *= dict((c, pr) for c, pr, _ in dist)[int(T[t])]
            visited.add(int(T[t]))
        p_oracle = float(np.prod(np.where(res["probs"][0][keep:] < 0, 1.0,
                                          res["probs"][0][keep:])))
        assert abs(p_oracle - float(p_exact)) <= 1e-12 * float(p_exact)
        # the replay agrees with the construction it replays
        cnt, prob = orc.replay_partial(xy, nn, nnd, tau, 1.0, 2.0, 11, it, ant, lb[0], 1.0, 4, T)
        assert cnt["kept"] == keep and cnt["invalid"] == 0 and cnt["hard_mismatch"] == 0
        np.testing.assert_allclose(prob[keep:], res["probs"][0][keep:], rtol=1e-15)
        checked += 1
    assert checked > 100


def test_plan_draws_have_the_stated_distributions():
    n, M, p = 1000, 37, 0.95
    S, R, P = [], [], []
    for it in range(1, 41):
        for ant in range(250):
            s, part, r = orc.partial_plan(9, it, ant, n, p, M)
            S.append(s)
            R.append(r)
            P.append(part)
    S, R, P = np.array(S), np.array(R), np.array(P)
    assert S.min() >= 0 and S.max() < n and R.min() >= 1 and R.max() <= M
    assert stats.chisquare(np.bincount(S // 100, minlength=10)).pvalue > 1e-3
    assert stats.chisquare(np.bincount(R - 1, minlength=M)).pvalue > 1e-3
    share = P.mean()
    sd = np.sqrt(p * (1 - p) / len(P))
    assert abs(share - p) < 5 * sd
    assert not any(orc.partial_plan(9, 1, a, n, 0.0, M)[1] for a in range(200))
    assert all(orc.partial_plan(9, 1, a, n, 1.0, M)[1] for a in range(200))
    # the cap is clamped to [1, n - 1]
    assert max(orc.partial_plan(9, 2, a, 50, 1.0, 10**6)[2] for a in range(500)) <= 49
    assert min(orc.partial_plan(9, 2, a, 50, 1.0, 0)[2] for a in range(50)) == 1


def test_local_best_replaced_only_when_strictly_shorter():
    lb = np.arange(12, dtype=np.int32).reshape(3, 4)
    lbl = np.array([10, 20, 30], np.int64)
    tours = lb[:, ::-1].copy()
    lengths = np.array([9, 20, 31], np.int64)
    nb, nl = orc.update_local_best(lb, lbl, tours, lengths)
    np.testing.assert_array_equal(nb, np.stack([tours[0], lb[1], lb[2]]))
    np.testing.assert_array_equal(nl, [9, 20, 30])


# ---------------------------------------------------------------- local-best pheromone
def _tour_slots(nn, tour):
    """Boolean [n][k]: slots (i, r) whose edge {i, nn[i][r]} is an edge of the tour."""
    n, k = nn.shape
    nxt = np.empty(n, np.int64)
    prv = np.empty(n, np.int64)
    t = np.asarray(tour, np.int64)
    nxt[t] = np.roll(t, -1)
    prv[t] = np.roll(t, 1)
    return (nn == nxt[:, None]) | (nn == prv[:, None])


def test_local_best_pheromone_one_tour_closed_form():
    xy, nn, nnd, tau = _instance(300, 8, 21)
    lb, lbl = _local_bests(xy, nn, nnd, tau, 1, 3)
    t, q = orc.pheromone_local_best(nn, lb, lbl, 0.5, 0.25)
    assert q[0] == 2**32                       # the global best itself has weight 1
    on = _tour_slots(nn, lb[0])
    assert on.any() and not on.all()
    np.testing.assert_array_equal(t[on], np.float32(0.75))
    np.testing.assert_array_equal(t[~on], np.float32(0.5))


def test_local_best_pheromone_weights_and_order():
    xy, nn, nnd, tau = _instance(300, 8, 22)
    lb, lbl = _local_bests(xy, nn, nnd, tau, 6, 4)
    t, q = orc.pheromone_local_best(nn, lb, lbl, 1.0 / 299, 1.0 / 6, shift=40)
    Lg = int(lbl.min())
    for a in range(6):
        exact_q = Fraction(Lg * 2**40, int(lbl[a]))
        assert abs(q[a] - exact_q) <= 1 and q[a] <= 2**40
    assert q[int(np.argmin(lbl))] == 2**40
    # the sum over ants does not depend on their order (integer accumulation)
    perm = np.array([3, 0, 5, 1, 4, 2])
    t2, _ = orc.pheromone_local_best(nn, lb[perm], lbl[perm], 1.0 / 299, 1.0 / 6, shift=40)
    np.testing.assert_array_equal(t.view(np.uint32), t2.view(np.uint32))
    # slots on no local best keep the base level; the others are above it
    on = np.zeros_like(nn, bool)
    for a in range(6):
        on |= _tour_slots(nn, lb[a])
    np.testing.assert_array_equal(t[~on], np.float32(1.0 / 299))
    assert (t[on] > np.float32(1.0 / 299)).all()
    # an edge used by every local best at weight ~1 carries about base + delta * m
    assert t.max() <= np.float32(1.0 / 299 + 1.0) * (1 + 1e-6)
