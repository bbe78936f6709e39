"""Pins of the oracle's Independent Roulette sampler (Section 3: the next
city is the largest product of weight and an independent uniform).

P(candidate r wins) = integral over u in [0, 1] of prod_{s != r} min(1, w_r u / w_s):
the chance that every other product falls below w_r u.  The oracle's first
moves from a fixed city over many (ant, iteration) draws follow it
(chi-square); a dominant weight always wins; equal weights choose uniformly."""
import numpy as np
import pytest
from scipy import integrate, stats

import oracle as orc
from paper_1709_03187_amd import instances

IR = orc.SAMPLER_INDEPENDENT


def _ir_probabilities(w):
    w = np.asarray(w, np.float64)
    out = []
    for r in range(len(w)):
        f = lambda u, r=r: np.prod([min(1.0, w[r] * u / w[s]) for s in range(len(w)) if s != r])
        out.append(integrate.quad(f, 0.0, 1.0, epsabs=1e-12, epsrel=1e-10, limit=200)[0])
    return np.array(out)


def _weights_row(nn, nnd, tau, c):
    """FP64 weights tau * (1/max(d,1))^2 of city c's candidates (alpha 1, beta 2)."""
    d = np.maximum(nnd[c], 1).astype(np.float64)
    return tau[c].astype(np.float64) / (d * d)


def _first_moves(xy, nn, nnd, tau, city, draws):
    n = len(xy)
    counts = {}
    got = 0
    for it in range(draws):
        ants = np.arange(64)
        res = orc.construct_partial(xy, nn, nnd, tau, 1.0, 2.0, 13, it, ants,
                                    np.zeros((64, n), np.int32), 0.0, 1, sampler=IR)
        for a in range(64):
            T = res["tours"][a]
            if T[0] == city:
                counts[int(T[1])] = counts.get(int(T[1]), 0) + 1
                got += 1
    return counts, got


def test_first_move_follows_the_exact_distribution():
    xy = np.array([[0, 0], [3, 0], [0, 5], [-7, 1], [2, -9], [12, 12]], np.int32)
    k = 5
    nn, nnd = orc.knn_rows(xy, k)
    tau = np.array([[1.0, 2.0, 0.5, 1.5, 3.0]] * 6, np.float32)
    counts, got = _first_moves(xy, nn, nnd, tau, 0, 300)
    assert got > 2000
    p = _ir_probabilities(_weights_row(nn, nnd, tau, 0))
    np.testing.assert_allclose(p.sum(), 1.0, atol=1e-9)
    obs = np.array([counts.get(int(j), 0) for j in nn[0]])
    chi = stats.chisquare(obs, p * got)
    assert chi.pvalue > 1e-3, (obs, p * got)
    # it differs from the roulette of Eq. 1 (probabilities proportional to w)
    w = _weights_row(nn, nnd, tau, 0)
    assert np.abs(p - w / w.sum()).max() > 0.05


def test_equal_weights_choose_uniformly_and_dominant_weight_always_wins():
    xy = np.array([[0, 0], [10, 0], [0, 10], [-10, 0], [0, -10], [50, 50]], np.int32)
    nn, nnd = orc.knn_rows(xy, 4)
    tau = np.ones((6, 4), np.float32)                 # four candidates at distance 10
    counts, got = _first_moves(xy, nn, nnd, tau, 0, 200)
    obs = np.array([counts.get(int(j), 0) for j in nn[0]])
    assert stats.chisquare(obs).pvalue > 1e-3
    tau2 = tau.copy()
    tau2[0, 2] = 1e9
    counts2, got2 = _first_moves(xy, nn, nnd, tau2, 0, 60)
    assert counts2 == {int(nn[0, 2]): got2}


def test_independent_roulette_tours_are_valid_and_replay_clean():
    xy = instances.uniform_coords(400, 3, hi=100_000)
    nn, nnd = orc.knn_rows(xy, 8)
    rng = np.random.default_rng(1)
    tau = rng.uniform(0.5, 2.0, (400, 8)).astype(np.float32)
    res = orc.construct_partial(xy, nn, nnd, tau, 1.0, 2.0, 5, 2, np.arange(8),
                                np.zeros((8, 400), np.int32), 0.0, 1, sampler=IR)
    for a in range(8):
        T = res["tours"][a]
        assert sorted(T) == list(range(400))
        assert res["lengths"][a] == orc.tour_length(xy, T)
        cnt, _ = orc.replay_partial(xy, nn, nnd, tau, 1.0, 2.0, 5, 2, a, np.zeros(400, np.int32),
                                    0.0, 1, T, sampler=IR)
        assert cnt["hard_mismatch"] == 0 and cnt["invalid"] == 0 and cnt["fallback_mismatch"] == 0
    # the roulette and the independent sampler give different tours from the same draws
    rou = orc.construct_partial(xy, nn, nnd, tau, 1.0, 2.0, 5, 2, np.arange(8),
                                np.zeros((8, 400), np.int32), 0.0, 1)
    assert not np.array_equal(rou["tours"], res["tours"])
    np.testing.assert_array_equal(rou["tours"][:, 0], res["tours"][:, 0])   # same start cities
