"""Seeded synthetic TSP instances shaped like the paper's workloads.

The paper evaluates on TSPLIB instances of 442-2,392 cities (Section 4,
Tables 1-7) and on art instances of 100K-200K cities (Section 5, Table 8).
Neither dataset is available here, so these generators stand in for them:
uniform random integer points for the TSPLIB scale and Gaussian clusters of
uneven density for the large art instances.

This module only produces inputs (integer coordinates, instance sizes).  It
holds none of the method's arithmetic and is the one piece of code shared by
the CPU oracle's tests and the GPU path's tests and benchmark.  Random words
come from numpy's Philox bit generator keyed by the seed; only its raw 64-bit
output is used, so the stream does not depend on numpy's distribution code.
"""
from __future__ import annotations

import math

import numpy as np

COORD_MAX = 10**6


def _raw(seed: int, tag: int, count: int) -> np.ndarray:
    """`count` raw uint64 words from the Philox stream keyed by (seed, tag)."""
    bg = np.random.Philox(key=np.array([seed & (2**64 - 1), tag], dtype=np.uint64))
    return bg.random_raw(count).astype(np.uint64)


def _words32(seed: int, tag: int, count: int) -> np.ndarray:
    """`count` uint32 words (low half first) from the (seed, tag) stream."""
    raw = _raw(seed, tag, (count + 1) // 2)
    out = np.empty(2 * raw.size, dtype=np.uint64)
    out[0::2] = raw & np.uint64(0xFFFFFFFF)
    out[1::2] = raw >> np.uint64(32)
    return out[:count]


def uniform_coords(n: int, seed: int, hi: int = COORD_MAX, tag: int = 1) -> np.ndarray:
    """n points with integer coordinates uniform on the closed square [0, hi]^2.

    Each coordinate is (w * (hi + 1)) >> 32 for a 32-bit word w.
    Returns int32 [n, 2] (x, y pairs)."""
    w = _words32(seed, tag, 2 * n)
    v = (w * np.uint64(hi + 1)) >> np.uint64(32)
    return v.astype(np.int32).reshape(n, 2)


def clustered_coords(n: int, seed: int, clusters: int = 100, sigma: float = 1.0e4,
                     hi: int = COORD_MAX, tag: int = 1) -> np.ndarray:
    """n points in `clusters` isotropic Gaussian clusters.

    Centres are uniform integers in [0, hi]^2; city i belongs to cluster
    i mod `clusters`; offsets are Box-Muller normals (FP64) scaled by sigma and
    the result is rounded half-to-even.  Points are not clamped to the square.
    Returns int32 [n, 2]."""
    cw = _words32(seed, tag, 2 * clusters)
    centres = ((cw * np.uint64(hi + 1)) >> np.uint64(32)).astype(np.float64).reshape(clusters, 2)
    raw = _raw(seed, tag + 1, 2 * n)
    u = (raw >> np.uint64(11)).astype(np.float64) * 2.0**-53      # [0, 1)
    u1, u2 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log1p(-u1))                           # log(1 - u1), u1 < 1
    ang = 2.0 * math.pi * u2
    c = np.arange(n) % clusters
    x = np.rint(centres[c, 0] + sigma * rad * np.cos(ang))
    y = np.rint(centres[c, 1] + sigma * rad * np.sin(ang))
    return np.stack([x, y], axis=1).astype(np.int32)


def batched_sizes(count: int, seed: int, lo: int = 100, hi: int = 5000, tag: int = 7) -> np.ndarray:
    """Instance sizes drawn log-uniform in [lo, hi]: round(exp(ln lo + u ln(hi/lo)))."""
    raw = _raw(seed, tag, count)
    u = (raw >> np.uint64(11)).astype(np.float64) * 2.0**-53
    n = np.rint(np.exp(math.log(lo) + u * math.log(hi / lo))).astype(np.int64)
    return np.clip(n, lo, hi)


def batched_coords(sizes: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Concatenated uniform instances: (xy int32 [sum n, 2], offsets int64 [B+1])."""
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    xy = np.empty((int(offsets[-1]), 2), dtype=np.int32)
    for b, nb in enumerate(sizes):
        xy[offsets[b]:offsets[b + 1]] = uniform_coords(int(nb), seed, tag=1000 + b)
    return xy, offsets


# The five workload configurations (sizes, colony parameters, seeds).
CONFIGS = {
    "c1": dict(kind="uniform", n=1000, m=32, k=10, alpha=1.0, beta=2.0, rho=0.1,
               iterations=10, seed=1),
    "c2": dict(kind="uniform", n=20000, m=256, k=16, alpha=1.0, beta=2.0, rho=0.1,
               iterations=50, seed=2),
    "c3": dict(kind="clustered", n=200000, m=1024, k=16, alpha=1.0, beta=2.0, rho=0.1,
               iterations=20, seed=3, clusters=100, sigma=1.0e4),
    "c4": dict(kind="batched", instances=4096, n_lo=100, n_hi=5000, m=64, k=12,
               alpha=1.0, beta=2.0, rho=0.1, iterations=30, seed=4),
}


def make_coords(name: str) -> np.ndarray:
    """Coordinates of a single-instance config (c1, c2, c3)."""
    cfg = CONFIGS[name]
    if cfg["kind"] == "uniform":
        return uniform_coords(cfg["n"], cfg["seed"])
    if cfg["kind"] == "clustered":
        return clustered_coords(cfg["n"], cfg["seed"], cfg["clusters"], cfg["sigma"])
    raise ValueError(f"{name} is not a single-instance config")


def make_batched(name: str = "c4", count: int | None = None):
    """(xy, offsets, sizes) of the batched config, optionally truncated to `count` instances."""
    cfg = CONFIGS[name]
    sizes = batched_sizes(cfg["instances"], cfg["seed"], cfg["n_lo"], cfg["n_hi"])
    if count is not None:
        sizes = sizes[:count]
    xy, offsets = batched_coords(sizes, cfg["seed"])
    return xy, offsets, sizes


def _uniform01(seed: int, tag: int, count: int) -> np.ndarray:
    """`count` FP64 uniforms in [0, 1) with 53 random bits each."""
    return (_raw(seed, tag, count) >> np.uint64(11)).astype(np.float64) * 2.0**-53


# Block (offset, size, half-width) of the edge-scoring network's parameters,
# in the order W1 [64][8], b1, W2 [64][64], b2, W3 [64], b3; the half-widths
# are the uniform He/Glorot ranges sqrt(6 / fan_in), sqrt(3 / fan_in).
MLP_BLOCKS = ((0, 512, math.sqrt(6 / 8)), (512, 64, 0.1), (576, 4096, math.sqrt(6 / 64)),
              (4672, 64, 0.1), (4736, 64, math.sqrt(3 / 64)), (4800, 1, 0.1))
MLP_PARAMS = 4801


def mlp_parameters(seed: int, tag: int = 50) -> np.ndarray:
    """Initial FP32 parameters of the edge-scoring network, uniform per block."""
    u = _uniform01(seed, tag, MLP_PARAMS)
    theta = np.empty(MLP_PARAMS, np.float64)
    for off, size, half in MLP_BLOCKS:
        theta[off:off + size] = (2.0 * u[off:off + size] - 1.0) * half
    return theta.astype(np.float32)


def mlp_edge_batch(E: int, seed: int, positive: float = 0.15, tag: int = 60):
    """Synthetic network inputs: FP32 features [E, 8] in the ranges the edge
    features take (ratios >= 1 and <= 1, ranks and rev in [0, 1], a unit
    direction, local radii around 1) and uint8 labels with P(1) = positive."""
    u = _uniform01(seed, tag, 9 * E).reshape(E, 9)
    X = np.empty((E, 8), np.float64)
    X[:, 0] = 1.0 + 7.0 * u[:, 0]
    X[:, 1] = u[:, 1]
    X[:, 2] = np.floor(16.0 * u[:, 2]) / 15.0
    X[:, 3] = np.where(u[:, 3] < 0.3, 1.0, u[:, 3])
    ang = 2.0 * math.pi * u[:, 4]
    X[:, 4] = np.cos(ang)
    X[:, 5] = np.sin(ang)
    X[:, 6] = 0.3 + 2.7 * u[:, 5]
    X[:, 7] = 0.3 + 2.7 * u[:, 6]
    y = (u[:, 8] < positive).astype(np.uint8)
    return X.astype(np.float32), y


def mlp_dyadic_batch(E: int, seed: int, positive: float = 0.15, tag: int = 70):
    """Parameters, features and labels on coarse dyadic grids: features
    j/8 in [0, 2), W1 j/16 and b1 j/128 in [-1/2, 1/2], W2, W3 j/8 in
    [-1/2, 1/2], b2 j/1024, b3 j/8192 in [-1/2, 1/2].  Products and partial
    sums of the network then need few enough bits that FP32 holds them
    exactly for the magnitudes these draws produce."""
    u = _uniform01(seed, tag, MLP_PARAMS + 9 * E)
    def grid(v, denom, half):
        return np.floor(v * (2 * half * denom + 1)) / denom - half
    t = np.empty(MLP_PARAMS, np.float64)
    blocks = ((0, 512, 16), (512, 64, 128), (576, 4096, 8), (4672, 64, 1024), (4736, 64, 8),
              (4800, 1, 8192))
    for off, size, denom in blocks:
        t[off:off + size] = grid(u[off:off + size], denom, 0.5)
    w = u[MLP_PARAMS:].reshape(E, 9)
    X = np.floor(w[:, :8] * 16) / 8
    y = (w[:, 8] < positive).astype(np.uint8)
    return t.astype(np.float32), X.astype(np.float32), y
