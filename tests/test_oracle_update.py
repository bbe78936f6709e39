"""Pins for the oracle's pheromone update: evaporation (Eq. 2) and the all-ant
deposit 1/C^k (Eq. 3-4) in int64 fixed point, merged with one FP32 rounding."""
import numpy as np
import pytest

from paper_1709_03187_amd import instances


def colony(orc, n=400, k=10, m=12, seed=5):
    xy = instances.uniform_coords(n, seed)
    nn, nnd = orc.knn_rows(xy, k)
    tau = np.full((n, k), orc.tau0(n, orc.nn_tour(xy, nn, nnd)[1]), np.float32)
    res = orc.construct(xy, nn, nnd, tau, 1.0, 2.0, seed=seed, iteration=0, ants=range(m))
    return xy, nn, nnd, tau, res


def test_pure_evaporation_closed_form(orc):
    # shift = 0 gives q = floor(1 / L) = 0: no deposit, tau_t = fl32(tau_{t-1} * f)
    xy, nn, nnd, tau, res = colony(orc)
    rho = 0.1
    f32 = np.float32(1.0 - rho)
    t_or, t_np = tau.copy(), tau.copy()
    for t in range(1, 60):
        t_or = orc.update(nn, t_or, res["tours"], res["lengths"], rho, shift=0)
        t_np = (t_np * f32).astype(np.float32)
        np.testing.assert_array_equal(t_or, t_np)
        closed = float(tau[0, 0]) * (1.0 - rho) ** t
        bound = (1 + 2.0**-24) ** (2 * t) - 1
        assert abs(float(t_or[0, 0]) - closed) <= bound * closed


def ref_acc(nn, tours, lengths, shift):
    """acc[i][r] = sum over ants whose tour uses edge {i, nn[i][r]} of floor(2^shift / L)."""
    n, k = nn.shape
    acc = np.zeros((n, k), np.int64)
    for a in range(tours.shape[0]):
        T = tours[a]
        edges = set()
        for t in range(n):
            i, j = int(T[t]), int(T[(t + 1) % n])
            edges.add((min(i, j), max(i, j)))
        q = (1 << shift) // int(lengths[a])
        for i in range(n):
            for r in range(k):
                j = int(nn[i, r])
                if (min(i, j), max(i, j)) in edges:
                    acc[i, r] += q
    return acc


def test_deposit_against_edge_sets(orc):
    xy, nn, nnd, tau, res = colony(orc, n=150, k=6, m=6)
    acc = orc.deposit(nn, res["tours"], res["lengths"], 32)
    np.testing.assert_array_equal(acc, ref_acc(nn, res["tours"], res["lengths"], 32))


def test_deposit_closing_edge(orc):
    # points on a circle, tours that walk around it from different starts: every
    # tour edge, the closing one included, joins neighbours on the circle
    n, k = 60, 4
    ang = 2 * np.pi * np.arange(n) / n
    xy = np.stack([np.rint(1e5 * np.cos(ang)), np.rint(1e5 * np.sin(ang))], 1).astype(np.int32)
    nn, nnd = orc.knn_rows(xy, k)
    tours = np.stack([np.roll(np.arange(n), -s) for s in (0, 7, 59)]).astype(np.int32)
    tours[2] = tours[2][::-1]
    lengths = np.array([orc.tour_length(xy, t) for t in tours], np.int64)
    acc = orc.deposit(nn, tours, lengths, 32)
    np.testing.assert_array_equal(acc, ref_acc(nn, tours, lengths, 32))
    q = sum((1 << 32) // int(L) for L in lengths)
    # both circle neighbours are candidates of every city, each edge in every tour
    for i in range(n):
        for r in range(k):
            j = int(nn[i, r])
            assert acc[i, r] == (q if (j - i) % n in (1, n - 1) else 0)


def test_deposit_conservation_and_symmetry(orc):
    xy, nn, nnd, tau, res = colony(orc, n=600, k=8, m=10)
    acc = orc.deposit(nn, res["tours"], res["lengths"], 32)
    n, k = nn.shape
    cand = {(i, int(nn[i, r])) for i in range(n) for r in range(k)}
    total = 0
    for a in range(10):
        T = res["tours"][a]
        hits = sum(((int(T[t]), int(T[(t + 1) % n])) in cand) +
                   ((int(T[(t + 1) % n]), int(T[t])) in cand) for t in range(n))
        total += ((1 << 32) // int(res["lengths"][a])) * hits
    assert acc.sum() == total
    rv = orc.rev(nn)
    for i in range(n):
        for r in range(k):
            if rv[i, r] >= 0:
                assert acc[i, r] == acc[nn[i, r], rv[i, r]]


@pytest.mark.parametrize("rho,shift", [(0.1, 32), (0.5, 40), (1.0, 32), (0.02, 20)])
def test_merge_bit_exact_numpy_float32(orc, rho, shift):
    xy, nn, nnd, tau, res = colony(orc, n=500, k=10, m=16)
    rng = np.random.default_rng(2)
    tau = (tau * rng.uniform(0.5, 2.0, size=tau.shape)).astype(np.float32)
    acc = orc.deposit(nn, res["tours"], res["lengths"], shift)
    got = orc.update(nn, tau, res["tours"], res["lengths"], rho, shift)
    evap = tau * np.float32(1.0 - rho)
    dep = acc.astype(np.float32) * np.float32(2.0**-shift)
    np.testing.assert_array_equal(got, (evap + dep).astype(np.float32))
    if rho == 1.0:
        np.testing.assert_array_equal(got, dep)


def test_run_best_tracking_and_determinism(orc):
    xy = instances.uniform_coords(300, 1)
    r1 = orc.run(xy, m=8, k=8, alpha=1.0, beta=2.0, rho=0.1, iterations=5, seed=1, threads=1)
    r2 = orc.run(xy, m=8, k=8, alpha=1.0, beta=2.0, rho=0.1, iterations=5, seed=1, threads=8)
    np.testing.assert_array_equal(r1["best_tour"], r2["best_tour"])
    np.testing.assert_array_equal(r1["tau"], r2["tau"])
    assert r1["best_len"] == orc.tour_length(xy, r1["best_tour"])
    nn, nnd = orc.knn_rows(xy, 8)
    L_nn = orc.nn_tour(xy, nn, nnd)[1]
    assert r1["best_len"] == min(L_nn, int(r1["iter_best"].min()))
    assert np.array_equal(np.sort(r1["best_tour"]), np.arange(300))


def test_deposit_threads_do_not_change_the_sums(orc):
    """Threads over groups of ants give the same exact int64 sums as one thread."""
    xy = instances.uniform_coords(600, 77)
    nn, _ = orc.knn_rows(xy, 9)
    rng = np.random.default_rng(5)
    tours = np.stack([rng.permutation(600) for _ in range(70)]).astype(np.int32)
    tours[:10] = tours[0]                       # shared edges across thread groups
    lengths = rng.integers(10**5, 10**7, 70)
    one = orc.deposit(nn, tours, lengths, 32, threads=1)
    for t in (2, 3, 16, 70):
        np.testing.assert_array_equal(orc.deposit(nn, tours, lengths, 32, threads=t), one)
    tau = np.full((600, 9), np.float32(1e-9))
    np.testing.assert_array_equal(orc.update(nn, tau, tours, lengths, 0.1, 32, threads=1),
                                  orc.update(nn, tau, tours, lengths, 0.1, 32, threads=7))
