"""Pins for the oracle's candidate lists (k smallest (d, j) per city; the
candidate-list idea of Section 6) and the reverse-slot table."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1709_03187_amd import instances
from tests._refs import knn_lexsort, nint_matrix


@pytest.mark.parametrize("n,k,span,seed", [(200, 10, 10**6, 1), (300, 16, 40, 2),
                                           (64, 63, 5, 3), (1000, 12, 10**6, 4)])
def test_knn_vs_lexsort(orc, n, k, span, seed):
    # small spans force many equal distances and coincident points
    xy = instances.uniform_coords(n, seed, hi=span)
    nn, nnd = orc.knn_rows(xy, k)
    rn, rd = knn_lexsort(xy, k)
    np.testing.assert_array_equal(nnd, rd)
    np.testing.assert_array_equal(nn, rn)


def test_knn_vs_ckdtree(orc):
    xy = instances.uniform_coords(4000, 9)
    k = 16
    rows = np.arange(0, 4000, 7, dtype=np.int32)
    nn, nnd = orc.knn_rows(xy, k, rows)
    tree = cKDTree(xy.astype(np.float64))
    _, idx = tree.query(xy[rows].astype(np.float64), k=k + 12)
    D = nint_matrix(xy, rows)
    checked = 0
    for q, i in enumerate(rows):
        cand = [int(j) for j in idx[q] if j != i]
        keys = sorted((int(D[q][j]), j) for j in cand)
        # the list is decided when the farthest returned neighbour is beyond the k-th distance
        if keys[-1][0] <= keys[k - 1][0]:
            continue
        assert [j for _, j in keys[:k]] == list(nn[q])
        assert [d for d, _ in keys[:k]] == list(nnd[q])
        checked += 1
    assert checked > 0.95 * len(rows)


def test_rev(orc):
    xy = instances.uniform_coords(500, 3, hi=300)
    nn, _ = orc.knn_rows(xy, 8)
    rv = orc.rev(nn)
    for i in range(500):
        for r in range(8):
            j = nn[i, r]
            hit = np.nonzero(nn[j] == i)[0]
            assert rv[i, r] == (hit[0] if len(hit) else -1)


def test_knn_threaded_equals_serial(orc):
    xy = instances.clustered_coords(3000, 5, clusters=7, sigma=2e4)
    a = orc.knn_rows(xy, 12)
    b = orc.knn_rows(xy, 12, threads=5)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
