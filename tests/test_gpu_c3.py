"""GPU parity at full size: n = 200,000 clustered cities, m = 1,024 ants,
k = 16 -- the launch configuration the benchmark times.  The oracle builds its
own candidate lists (threads over rows) and NN tour; it replays a sample of
ants step by step and recomputes the pheromone update of all 1,024 tours
bit-exactly; properties (permutation, exact length, slot records) are checked
for every ant."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import check_tours, colony, require_gpu, say, threads, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    require_gpu()
    cfg = instances.CONFIGS["c3"]
    xy = instances.make_coords("c3")
    say(f"[c3] oracle candidate lists, {threads()} threads")
    nn, nnd = orc.knn_rows(xy, cfg["k"], threads=threads())
    return cfg, xy, nn, nnd


def tour_lengths_np(xy, tours):
    a = xy[tours].astype(np.int64)
    b = xy[np.roll(tours, -1, axis=1)].astype(np.int64)
    s = ((a - b) ** 2).sum(-1)
    r = np.floor(np.sqrt(s.astype(np.float64))).astype(np.int64)
    r -= (r * r > s)
    r += ((r + 1) * (r + 1) <= s)
    return np.where(s - r * r > r, r + 1, r).sum(1)


def test_c3_candidates_init_construct_update(c3):
    import torch
    cfg, xy, nn, nnd = c3
    n, m, k = cfg["n"], cfg["m"], cfg["k"]
    say("[c3] GPU set-up")
    col = colony(xy, k=k, m=m, alpha=cfg["alpha"], beta=cfg["beta"], rho=cfg["rho"],
                 seed=cfg["seed"], want_prob=True)
    col.setup()
    np.testing.assert_array_equal(to_np(col.nn), nn)
    np.testing.assert_array_equal(to_np(col.nnd), nnd)
    np.testing.assert_array_equal(to_np(col.rev), orc.rev(nn))
    say("[c3] oracle NN tour")
    tour, L = orc.nn_tour(xy, nn, nnd)
    np.testing.assert_array_equal(to_np(col.nn_tour), tour)
    assert col.L_nn == L
    tau = np.full((n, k), orc.tau0(n, L), np.float32)
    np.testing.assert_array_equal(to_np(col.tau), tau)

    say("[c3] construct iteration 0")
    col.construct(0)
    torch.cuda.synchronize()
    tours, lengths, slots = to_np(col.tours), to_np(col.lengths), to_np(col.slots)
    probs = to_np(col.step_prob)
    # properties of every ant
    assert np.array_equal(np.sort(tours, axis=1), np.broadcast_to(np.arange(n), tours.shape))
    np.testing.assert_array_equal(lengths, tour_lengths_np(xy, tours))
    assert np.all(slots[:, 0] == 255)
    cand = slots[:, 1:] != 255
    prev = tours[:, :-1][cand]
    np.testing.assert_array_equal(nn[prev, slots[:, 1:][cand]], tours[:, 1:][cand])
    # step-by-step replay of a sample of ants
    sample = np.array([0, 1, 511, 1023, 77, 300, 640, 999][:max(2, min(8, threads()))])
    say(f"[c3] oracle replay of ants {list(sample)}")
    tot = check_tours(xy, nn, nnd, tau, cfg["alpha"], cfg["beta"], cfg["seed"], 0,
                      tours[sample], lengths[sample], slots[sample], probs[sample], sample,
                      label="c3")
    say(f"[c3] replay totals {tot}")
    say("[c3] update")
    col.update()
    torch.cuda.synchronize()
    ref = orc.update(nn, tau, tours, lengths, cfg["rho"], 32)
    np.testing.assert_array_equal(to_np(col.tau), ref)
