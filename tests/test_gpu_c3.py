"""GPU parity at full size: n = 200,000 clustered cities, m = 1,024 ants,
k = 16, in the launch configuration the benchmark times (the production
construction kernel, which keeps no step-probability record).

Set-up: candidate lists, reverse slots and the NN tour are compared with the
oracle's.  Then iterations 0 .. ITERS-1 run as in the benchmark (construct,
best tracking, update) and each is checked:
- every one of the 1,024 tours: a permutation, its exact length, its slot
  records pointing at the city taken;
- the probability-recording variant of the kernel, run on the same pheromone,
  builds exactly the same tours, and its step probabilities of the replayed
  ants agree with the oracle's to 1e-5;
- the oracle replays a fixed sample of 32 ants step by step (all 1,024 at the
  last iteration, the benchmark's first timed one);
- the best so far equals the shortest tour seen (or the NN tour);
- the pheromone after the update is bit-exact with the oracle's update of the
  GPU's tours (so the next iteration starts from the same pheromone).
Fallback moves are checked with the oracle's sweep along x, which returns the
same city as its brute-force search (pinned in test_oracle_fallback_nn.py)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import check_tours, require_gpu, say, threads, to_np

pytestmark = pytest.mark.gpu

ITERS = 6                    # iterations 0..5; the benchmark times from iteration 5 on
SAMPLE = np.array(sorted({0, 1, 2, 3, 77, 128, 255, 256, 300, 333, 384, 400, 444, 500, 511,
                          512, 555, 600, 640, 666, 700, 767, 768, 800, 888, 900, 960, 999,
                          1000, 1010, 1022, 1023}))


@pytest.fixture(scope="module")
def c3():
    require_gpu()
    import torch
    import paper_1709_03187_amd as aco
    assert len(SAMPLE) == 32
    cfg = instances.CONFIGS["c3"]
    xy = instances.make_coords("c3")
    n, m, k = cfg["n"], cfg["m"], cfg["k"]
    say(f"[c3] oracle candidate lists, {threads()} threads")
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    col = aco.Colony(xy=xy, k=k, m=m, alpha=cfg["alpha"], beta=cfg["beta"], rho=cfg["rho"],
                     seed=cfg["seed"], device="cuda:0")
    # second set of outputs for the probability-recording kernel variant
    side = dict(tours=torch.empty((m, n), dtype=torch.int32, device="cuda:0"),
                lengths=torch.empty(m, dtype=torch.int64, device="cuda:0"),
                slots=torch.empty((m, n), dtype=torch.uint8, device="cuda:0"),
                prob=torch.empty((m, n), dtype=torch.float32, device="cuda:0"))
    state = dict(cfg=cfg, xy=xy, nn=nn, nnd=nnd, col=col, side=side, iter_best=[],
                 sweep=orc.x_sweep_index(xy))
    return state


def test_c3_setup(c3):
    import torch
    col, xy, nn, nnd = c3["col"], c3["xy"], c3["nn"], c3["nnd"]
    n, k = len(xy), nn.shape[1]
    say("[c3] GPU set-up")
    col.setup()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(col.nn), nn)
    np.testing.assert_array_equal(to_np(col.nnd), nnd)
    np.testing.assert_array_equal(to_np(col.rev), orc.rev(nn))
    say("[c3] oracle NN tour")
    tour, L = orc.nn_tour(xy, nn, nnd)
    np.testing.assert_array_equal(to_np(col.nn_tour), tour)
    assert col.L_nn == L
    tau = np.full((n, k), orc.tau0(n, L), np.float32)
    np.testing.assert_array_equal(to_np(col.tau), tau)
    c3["tau"] = tau
    c3["L_nn"] = L


def _lengths(xy, tours):
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        return np.array(list(ex.map(lambda t: orc.tour_length(xy, t), tours)), np.int64)


@pytest.mark.parametrize("it", range(ITERS))
def test_c3_iteration(c3, it, report):
    import torch
    import paper_1709_03187_amd as aco
    assert "tau" in c3, "set-up test did not run"
    cfg, col, side, xy, nn, nnd = c3["cfg"], c3["col"], c3["side"], c3["xy"], c3["nn"], c3["nnd"]
    n, m, k = cfg["n"], cfg["m"], cfg["k"]
    tau = c3["tau"]
    np.testing.assert_array_equal(to_np(col.tau), tau, err_msg=f"tau before iteration {it}")

    say(f"[c3] iteration {it}: production construction, probability-recording variant")
    col.construct(it)
    aco.aco_construct_tours(col.xy, n, k, col.nn, col.nnd, col.eta_b, col.grid, col.tau, m, 0,
                            cfg["alpha"], cfg["seed"], it, side["tours"], side["lengths"],
                            side["slots"], side["prob"], col.cws)
    ib = torch.empty(1, dtype=torch.int64, device="cuda:0")
    col.track_best(ib)
    torch.cuda.synchronize()
    tours, lengths, slots = to_np(col.tours), to_np(col.lengths), to_np(col.slots)
    assert np.array_equal(to_np(side["tours"]), tours), "probability variant built other tours"
    assert np.array_equal(to_np(side["lengths"]), lengths)
    assert np.array_equal(to_np(side["slots"]), slots)

    say(f"[c3] iteration {it}: properties of all {m} tours")
    seen = np.zeros((m, n), np.bool_)
    seen[np.arange(m)[:, None], tours] = True
    assert seen.all(), "a tour is not a permutation"
    del seen
    np.testing.assert_array_equal(lengths, _lengths(xy, tours))
    assert np.all(slots[:, 0] == 255)
    cand = slots[:, 1:] != 255
    prev = tours[:, :-1][cand]
    np.testing.assert_array_equal(nn[prev, slots[:, 1:][cand]], tours[:, 1:][cand])
    del cand, prev

    ants = np.arange(m) if it == ITERS - 1 else SAMPLE
    say(f"[c3] iteration {it}: oracle replay of {len(ants)} ants")
    probs = to_np(side["prob"][torch.as_tensor(ants, device="cuda:0")])
    tot = check_tours(xy, nn, nnd, tau, cfg["alpha"], cfg["beta"], cfg["seed"], it, tours[ants],
                      lengths[ants], slots[ants], probs, ants, label=f"c3 it {it}",
                      sweep=c3["sweep"])
    report(f"\n[c3] iteration {it}: oracle replayed {len(ants)} of {m} ants, {tot}")
    assert tot["steps"] == len(ants) * (n - 1)

    c3["iter_best"].append(int(lengths.min()))
    assert int(ib.item()) == int(lengths.min())
    assert int(col.best_len.item()) == min([c3["L_nn"]] + c3["iter_best"])

    say(f"[c3] iteration {it}: update")
    col.update()
    torch.cuda.synchronize()
    tau = orc.update(nn, tau, tours, lengths, cfg["rho"], 32, threads=threads())
    np.testing.assert_array_equal(to_np(col.tau), tau, err_msg=f"tau after iteration {it}")
    c3["tau"] = tau
    report(f"[c3] iteration {it}: all {m} tours valid with exact lengths; pheromone bit-exact "
           f"after the update (min {tau.min():.4g}, max {tau.max():.4g})")
