"""Pins for the oracle's tour construction (random proportional rule, Eq. 1,
with the nearest-unvisited fallback) against exact rational arithmetic,
exhaustive tour enumeration, closed-form special cases and invariants."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from paper_1709_03187_amd import instances
from tests._refs import nint_matrix


def small_instance(n, k, seed, span=1000, tau_lo=1e-6, tau_hi=1e-3):
    xy = instances.uniform_coords(n, seed, hi=span)
    pts = [tuple(map(int, p)) for p in xy]
    nn, nnd = exact.candidate_lists(pts, k)
    rng = np.random.default_rng(seed)
    tau = rng.uniform(tau_lo, tau_hi, size=(n, k)).astype(np.float32)
    return xy, pts, np.array(nn, np.int32), np.array(nnd, np.int32), tau


def test_exact_candidate_lists_agree_with_oracle(orc):
    xy, pts, nn, nnd, _ = small_instance(40, 7, 3, span=25)
    onn, onnd = orc.knn_rows(xy, 7)
    np.testing.assert_array_equal(onn, nn)
    np.testing.assert_array_equal(onnd, nnd)


@pytest.mark.parametrize("n,k,seed", [(12, 5, 1), (15, 3, 2), (10, 9, 3), (20, 2, 4)])
def test_step_probabilities_exact(orc, n, k, seed):
    xy, pts, nn, nnd, tau = small_instance(n, k, seed)
    res = orc.construct(xy, nn, nnd, tau, 1.0, 2.0, seed=77, iteration=0, ants=range(16),
                        want_slots=True, want_probs=True)
    for a in range(16):
        tour = res["tours"][a]
        visited = {int(tour[0])}
        u_words = [orc.draw(77, 0, a, t) for t in range(n)]
        assert tour[0] == (u_words[0] * n) >> 32
        for t in range(1, n):
            c = int(tour[t - 1])
            dist = exact.step_distribution(c, visited, pts, nn.tolist(), nnd.tolist(),
                                           tau.tolist(), 1, 2)
            j = int(tour[t])
            match = [(q, r) for (city, q, r) in dist if city == j]
            assert match, "oracle moved to a city with zero probability"
            q, r = match[0]
            if r < 0:
                assert res["probs"][a, t] == -1.0 and res["slots"][a, t] == -1
            else:
                assert res["slots"][a, t] == r
                assert abs(res["probs"][a, t] - float(q)) <= 1e-14 * float(q)
                # the roulette: u falls in j's cumulative interval (exactly, up to 1e-12)
                u = Fraction(u_words[t], 2**32)
                cum = Fraction(0)
                for city, qq, _ in dist:
                    if city == j:
                        assert cum - Fraction(1, 10**12) <= u < cum + qq + Fraction(1, 10**12)
                        break
                    cum += qq
            visited.add(j)


@pytest.mark.parametrize("n,k", [(5, 4), (6, 5), (6, 2), (7, 3)])
def test_enumeration_matches_replay_product(orc, n, k):
    xy, pts, nn, nnd, tau = small_instance(n, k, 100 + n * k)
    for start in range(n):
        dist = exact.tour_distribution(pts, nn.tolist(), nnd.tolist(), tau.tolist(), start)
        assert sum(dist.values()) == 1
        for tour, p in dist.items():
            # find an ant whose start is `start` (the replay checks the start city too)
            _, prob = orc.replay(xy, nn, nnd, tau, 1.0, 2.0, seed=5, iteration=0, ant=0,
                                 tour=np.array(tour, np.int32))
            steps = prob[1:]
            prod = float(np.prod(np.where(steps < 0, 1.0, steps)))
            assert abs(prod - float(p)) <= 1e-12 * float(p)


def chi2_against(probs: dict, counts: dict, total: int):
    """Chi-square statistic and dof with bins pooled to expected >= 5."""
    items = sorted(probs.items(), key=lambda kv: float(kv[1]))
    stat, dof, pool_e, pool_o = 0.0, 0, 0.0, 0
    for key, p in items:
        pool_e += float(p) * total
        pool_o += counts.get(key, 0)
        if pool_e >= 5:
            stat += (pool_o - pool_e) ** 2 / pool_e
            dof += 1
            pool_e, pool_o = 0.0, 0
    assert sum(counts.values()) == total
    assert set(counts) <= set(probs), "sampled a tour of probability zero"
    return stat, dof - 1


def chi2_crit(dof):
    # Wilson-Hilferty upper quantile at p ~ 1e-5 (z = 4.26)
    z = 4.26
    return dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3


@pytest.mark.parametrize("n,k,alpha,beta", [(5, 4, 1, 2), (6, 2, 1, 2), (5, 4, 0, 0)])
def test_sampling_distribution(orc, n, k, alpha, beta):
    xy, pts, nn, nnd, tau = small_instance(n, k, 40 + n + k)
    probs = {}
    for s in range(n):
        ps = exact.start_probability(s, n)
        for tour, p in exact.tour_distribution(pts, nn.tolist(), nnd.tolist(), tau.tolist(), s,
                                               alpha, beta).items():
            probs[tour] = ps * p
    assert sum(probs.values()) == 1
    A = 40_000
    res = orc.construct(xy, nn, nnd, tau, float(alpha), float(beta), seed=9, iteration=3,
                        ants=range(A))
    counts = {}
    for t in map(tuple, res["tours"].tolist()):
        counts[t] = counts.get(t, 0) + 1
    stat, dof = chi2_against(probs, counts, A)
    assert stat < chi2_crit(dof), (stat, dof)


def test_uniform_permutations_when_alpha_beta_zero():
    # alpha = beta = 0 and k = n - 1: every candidate has weight 1, so each
    # ordering of the other cities has probability 1/(n-1)!
    n = 6
    xy, pts, nn, nnd, tau = small_instance(n, n - 1, 8)
    dist = exact.tour_distribution(pts, nn.tolist(), nnd.tolist(), tau.tolist(), 2, 0, 0)
    assert len(dist) == math.factorial(n - 1)
    assert set(dist.values()) == {Fraction(1, math.factorial(n - 1))}


def test_large_beta_is_greedy(orc):
    # with beta = 60 the nearest unvisited candidate dominates: wherever the other
    # unvisited candidates carry less than 1e-9 of the weight, the move is the
    # greedy nearest-neighbour one; with no unvisited candidate it is the fallback
    n, k, beta = 300, 8, 60.0
    xy = instances.uniform_coords(n, 12)
    nn, nnd = orc.knn_rows(xy, k)
    tau = np.full((n, k), 1e-3, np.float32)
    res = orc.construct(xy, nn, nnd, tau, 1.0, beta, seed=3, iteration=0, ants=range(4))
    D = nint_matrix(xy)
    checked = 0
    for a in range(4):
        tour = res["tours"][a]
        vis = np.zeros(n, bool)
        vis[tour[0]] = True
        for t in range(1, n):
            c = tour[t - 1]
            un = np.nonzero(~vis)[0]
            greedy = un[np.lexsort((un, D[c][un]))[0]]
            ds = [int(nnd[c, r]) for r in range(k) if not vis[nn[c, r]]]
            if ds:
                rest = sum((ds[0] / d) ** beta for d in ds[1:]) if ds[0] > 0 else 1.0
                if rest < 1e-9:
                    assert tour[t] == greedy
                    checked += 1
            else:
                assert tour[t] == greedy
                checked += 1
            vis[tour[t]] = True
    assert checked > 0.5 * 4 * (n - 1)


@pytest.mark.parametrize("name_n,k", [(2000, 10), (3000, 16)])
def test_invariants_and_self_replay(orc, name_n, k):
    n = name_n
    xy = instances.uniform_coords(n, 31)
    nn, nnd = orc.knn_rows(xy, k)
    rng = np.random.default_rng(1)
    tau = rng.uniform(1e-9, 1e-8, size=(n, k)).astype(np.float32)
    res = orc.construct(xy, nn, nnd, tau, 1.0, 2.0, seed=4, iteration=2, ants=range(8),
                        want_slots=True, want_probs=True)
    D_len = lambda tour: orc.tour_length(xy, tour)
    for a in range(8):
        tour = res["tours"][a]
        assert np.array_equal(np.sort(tour), np.arange(n))
        assert tour[0] == orc.start_city(4, 2, a, n)
        assert res["lengths"][a] == D_len(tour)
        sl = res["slots"][a]
        assert res["fallbacks"][a] == int((sl[1:] < 0).sum())
        for t in range(1, n):
            if sl[t] >= 0:
                assert nn[tour[t - 1], sl[t]] == tour[t]
        counts, prob = orc.replay(xy, nn, nnd, tau, 1.0, 2.0, 4, 2, a, tour)
        assert counts["steps"] == n - 1
        assert counts["hard_mismatch"] == counts["fallback_mismatch"] == counts["invalid"] == 0
        assert counts["near_boundary_mismatch"] == 0
        np.testing.assert_array_equal(prob[1:], res["probs"][a, 1:])
