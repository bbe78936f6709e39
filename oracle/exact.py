"""Exact rational oracle for tiny instances -- TEST INFRASTRUCTURE ONLY.

Independent of `aco_oracle.c`: pure Python with `fractions.Fraction`, used
to pin the FP64 oracle.  With alpha = 1 and beta = 2 the weight of a
candidate edge, tau * (1/d)^2 (Section 2, Eq. 1 with eta = 1/d), is a
rational number when tau is a binary FP32 value and d an integer, so every
choice probability is an exact fraction.

Also enumerates every tour an ant can build on a tiny instance (n <= 7) with
its exact probability, which fixes the whole distribution the sampler must
reproduce.
"""
from __future__ import annotations

import math
from fractions import Fraction


def nint_dist(p, q) -> int:
    """nint of the Euclidean distance, by integer square root."""
    s = (p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2
    r = math.isqrt(s)
    # sqrt(s) >= r + 1/2  <=>  4s >= 4r^2 + 4r + 1  <=>  4s > 4r^2 + 4r (never equal)
    return r + 1 if 4 * s > 4 * r * r + 4 * r else r


def candidate_lists(pts, k):
    """k smallest (d, j), j != i, per city, by exhaustive sort."""
    n = len(pts)
    nn, nnd = [], []
    for i in range(n):
        keys = sorted((nint_dist(pts[i], pts[j]), j) for j in range(n) if j != i)[:k]
        nn.append([j for _, j in keys])
        nnd.append([d for d, _ in keys])
    return nn, nnd


def weight(tau_val, d, alpha: int = 1, beta: int = 2) -> Fraction:
    """tau^alpha * (1/max(d,1))^beta for integer alpha, beta >= 0, exactly."""
    t = Fraction(float(tau_val))
    e = Fraction(1, max(int(d), 1))
    return t ** alpha * e ** beta


def step_distribution(c, visited, pts, nn, nnd, tau, alpha=1, beta=2):
    """Exact distribution of the next city from c.

    Returns a list of (city, probability, slot) over unvisited candidates with
    positive weight; when there are none, the deterministic nearest unvisited
    city (smallest (d, j)) with probability 1 and slot -1."""
    w = []
    for r, j in enumerate(nn[c]):
        if j in visited:
            continue
        x = weight(tau[c][r], nnd[c][r], alpha, beta)
        if x > 0:
            w.append((j, x, r))
    S = sum(x for _, x, _ in w)
    if w and S > 0:
        return [(j, x / S, r) for j, x, r in w]
    n = len(pts)
    best = min((nint_dist(pts[c], pts[j]), j) for j in range(n) if j not in visited)
    return [(best[1], Fraction(1), -1)]


def start_probability(s: int, n: int) -> Fraction:
    """P(start = s) when start = (x * n) >> 32 for x uniform on 32-bit words:
    the number of x with s * 2^32 <= x * n < (s + 1) * 2^32, over 2^32."""
    lo = -((-s * 2**32) // n)          # ceil(s 2^32 / n)
    hi = -((-(s + 1) * 2**32) // n)
    return Fraction(hi - lo, 2**32)


def tour_distribution(pts, nn, nnd, tau, start, alpha=1, beta=2):
    """Every tour from `start` with its exact probability: dict tuple(tour) -> Fraction."""
    out = {}

    def rec(tour, visited, p):
        if len(tour) == len(pts):
            out[tuple(tour)] = out.get(tuple(tour), 0) + p
            return
        for j, q, _ in step_distribution(tour[-1], visited, pts, nn, nnd, tau, alpha, beta):
            visited.add(j)
            tour.append(j)
            rec(tour, visited, p * q)
            tour.pop()
            visited.remove(j)

    rec([start], {start}, Fraction(1))
    return out


def tour_length(pts, tour) -> int:
    n = len(tour)
    return sum(nint_dist(pts[tour[t]], pts[tour[(t + 1) % n]]) for t in range(n))
