"""Independent numpy references used to pin the CPU oracle (test helpers only)."""
import numpy as np


def nint_matrix(xy: np.ndarray, rows=None) -> np.ndarray:
    """nint Euclidean distances from `rows` to every city, exact for |coords| < 2^26."""
    xy = xy.astype(np.int64)
    src = xy if rows is None else xy[np.asarray(rows)]
    dx = src[:, None, 0] - xy[None, :, 0]
    dy = src[:, None, 1] - xy[None, :, 1]
    s = dx * dx + dy * dy
    r = np.floor(np.sqrt(s.astype(np.float64))).astype(np.int64)
    r -= (r * r > s)
    r += ((r + 1) * (r + 1) <= s)
    return np.where(s - r * r > r, r + 1, r)


def knn_lexsort(xy: np.ndarray, k: int, rows=None):
    """k smallest (d, j), j != i, by numpy lexsort over the full distance rows."""
    n = len(xy)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    D = nint_matrix(xy, rows)
    nn = np.empty((len(rows), k), np.int32)
    nnd = np.empty((len(rows), k), np.int32)
    idx = np.arange(n)
    for q, i in enumerate(rows):
        mask = idx != i
        js, ds = idx[mask], D[q][mask]
        order = np.lexsort((js, ds))[:k]
        nn[q], nnd[q] = js[order], ds[order]
    return nn, nnd
