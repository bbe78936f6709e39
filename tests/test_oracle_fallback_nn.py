"""Pins for the oracle's nearest-unvisited fallback and nearest-neighbour tour
(the deterministic (d, j) rule used when every candidate is visited, and the
tour that sets the initial pheromone 1/(n L_nn))."""
import numpy as np
import pytest

from paper_1709_03187_amd import instances
from tests._refs import nint_matrix


def test_fallback_two_pass_equals_plain_and_numpy(orc):
    rng = np.random.default_rng(0)
    for span in (3, 20, 10**6):
        xy = instances.uniform_coords(400, 21 + span, hi=span)
        D = nint_matrix(xy)
        for trial in range(200):
            vis = (rng.random(400) < rng.random()).astype(np.uint8)
            c = int(rng.integers(400))
            vis[c] = 1
            if vis.all():
                continue
            a = orc.nearest_unvisited(xy, c, vis)
            b = orc.nearest_unvisited(xy, c, vis, plain=True)
            un = np.nonzero(vis == 0)[0]
            ref = un[np.lexsort((un, D[c][un]))[0]]
            assert a == b == ref


@pytest.mark.parametrize("n,k,span", [(300, 5, 10**6), (500, 8, 30), (257, 3, 10**6),
                                      (65, 64, 7)])
def test_nn_tour_shortcut_equals_plain(orc, n, k, span):
    xy = instances.uniform_coords(n, n + k, hi=span)
    nn, nnd = orc.knn_rows(xy, k)
    t1, L1 = orc.nn_tour(xy, nn, nnd)
    t2, L2 = orc.nn_tour_plain(xy)
    np.testing.assert_array_equal(t1, t2)
    assert L1 == L2 == orc.tour_length(xy, t1)
    # numpy greedy walk
    D = nint_matrix(xy)
    vis = np.zeros(n, bool)
    c = 0
    vis[0] = True
    for t in range(1, n):
        un = np.nonzero(~vis)[0]
        j = un[np.lexsort((un, D[c][un]))[0]]
        assert t1[t] == j
        vis[j] = True
        c = j


def test_tau0(orc):
    assert orc.tau0(1000, 123456) == np.float32(1.0 / (1000.0 * 123456.0))
