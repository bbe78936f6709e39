"""GPU parity of PartialACO (Section 3.1, Algorithm 1; cap and probability of
partial modification, Section 4) against the CPU oracle.

Iteration 0 is a full construction whose tours become the local bests; each
later iteration every ant is replayed by the oracle from its own plan: the
kept part must be the planned segment of its local best, the rebuilt steps
follow the standard replay protocol (probabilities to 1e-5, choices equal
outside the 1e-6 window, fallbacks exact).  Local bests and the pheromone
update are compared exactly."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import (BOUNDARY_EPS, BOUNDARY_RATE, PROB_RTOL, colony, require_gpu, say,
                            threads)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def check_partial(xy, nn, nnd, tau, seed, it, lbest, p, M, tours, lengths, slots, probs,
                  ants, label):
    n, k = nn.shape
    tot = dict(steps=0, near=0, kept=0)
    for a in ants:
        T = tours[a]
        cnt, oprob = orc.replay_partial(xy, nn, nnd, tau, 1.0, 2.0, seed, it, a, lbest[a], p, M, T,
                                        boundary_eps=BOUNDARY_EPS)
        assert cnt["invalid"] == 0 and cnt["hard_mismatch"] == 0, (label, a, cnt)
        assert cnt["fallback_mismatch"] == 0, (label, a, cnt)
        keep = cnt["kept"] if cnt["kept"] < n else 1
        tot["steps"] += cnt["steps"]
        tot["near"] += cnt["near_boundary_mismatch"]
        tot["kept"] += cnt["kept"] if cnt["kept"] < n else 0
        assert np.array_equal(np.sort(T), np.arange(n)), (label, a)
        assert lengths[a] == orc.tour_length(xy, T), (label, a)
        sl, pr = slots[a], probs[a]
        assert (sl[:keep] == 255).all() and (pr[:keep] == 1.0).all(), (label, a)
        fb = sl[keep:] == 255
        assert np.array_equal(fb, oprob[keep:] < 0), (label, a)
        idx = np.nonzero(~fb)[0] + keep
        assert np.array_equal(nn[T[idx - 1], sl[idx]], T[idx]), (label, a)
        np.testing.assert_allclose(pr[idx], oprob[idx], rtol=PROB_RTOL, err_msg=f"{label} {a}")
        assert (pr[np.nonzero(fb)[0] + keep] == -1.0).all()
    assert tot["near"] <= BOUNDARY_RATE * max(tot["steps"], 1)
    return tot


def run_partial(xy, k, m, seed, schedule, label):
    """schedule: list of (p, M) for iterations 1, 2, ..."""
    col = colony(xy, k=k, m=m, seed=seed, want_prob=True)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    np.testing.assert_array_equal(_np(col.nn), nn)
    tau = _np(col.tau).copy()
    col.construct(0)
    col.update_local_best()
    tours, lengths = _np(col.tours), _np(col.lengths)
    lbest, lbest_len = orc.update_local_best(np.zeros_like(tours), np.full(m, 2**63 - 1),
                                             tours, lengths)
    np.testing.assert_array_equal(_np(col.lbest), lbest)
    col.update()
    tau = orc.update(nn, tau, tours, lengths, 0.1, 32)
    np.testing.assert_array_equal(_np(col.tau), tau)
    for it, (p, M) in enumerate(schedule, start=1):
        say(f"[partial] {label} iteration {it} p={p} M={M}")
        col.construct_partial(it, p, M)
        tours, lengths = _np(col.tours), _np(col.lengths)
        tot = check_partial(xy, nn, nnd, tau, seed, it, lbest, p, M, tours, lengths,
                            _np(col.slots), _np(col.step_prob), range(m), f"{label} it={it}")
        col.update_local_best()
        lbest, lbest_len = orc.update_local_best(lbest, lbest_len, tours, lengths)
        np.testing.assert_array_equal(_np(col.lbest), lbest)
        np.testing.assert_array_equal(_np(col.lbest_len), lbest_len)
        col.update()
        tau = orc.update(nn, tau, tours, lengths, 0.1, 32)
        np.testing.assert_array_equal(_np(col.tau), tau, err_msg=f"{label} it={it}")
        say(f"[partial] {label} it={it}: {tot}")
    return col


def test_partial_c1_with_cap_and_probability():
    cfg = instances.CONFIGS["c1"]
    run_partial(instances.make_coords("c1"), cfg["k"], cfg["m"], 1,
                [(0.95, 100), (0.95, 100), (1.0, 999), (0.5, 10)], "c1")


def test_partial_clustered_small_cap():
    xy = instances.clustered_coords(3000, 17, clusters=12, sigma=2000.0)
    run_partial(xy, 16, 16, 5, [(1.0, 30), (1.0, 30), (0.95, 300)], "clustered")


def test_probability_zero_equals_full_construction():
    import torch
    xy = instances.make_coords("c1")
    col = colony(xy, k=10, m=16, seed=3, want_prob=True)
    col.setup()
    col.construct(0)
    col.update_local_best()
    col.construct(1)
    full = [_np(t).copy() for t in (col.tours, col.lengths, col.slots, col.step_prob)]
    col.construct_partial(1, 0.0, 50)
    part = [_np(t) for t in (col.tours, col.lengths, col.slots, col.step_prob)]
    for a, b in zip(full, part):
        np.testing.assert_array_equal(a, b)
    torch.cuda.synchronize()


def test_one_rebuilt_city_rotates_the_local_best():
    xy = instances.make_coords("c1")
    col = colony(xy, k=10, m=8, seed=4)
    col.setup()
    col.construct(0)
    col.update_local_best()
    lb = _np(col.lbest).copy()
    lb_len = _np(col.lbest_len).copy()
    col.construct_partial(1, 1.0, 1)
    tours, lengths = _np(col.tours), _np(col.lengths)
    for a in range(8):
        s, partial, r = orc.partial_plan(4, 1, a, len(xy), 1.0, 1)
        np.testing.assert_array_equal(tours[a], np.roll(lb[a], -s))
        # the length summed over the kept segment and the closing edge is the local best's
        assert lengths[a] == lb_len[a] == orc.tour_length(xy, tours[a])


def test_partial_full_size_sample():
    """200,000 clustered cities, m = 1,024, the 1% cap: every tour is checked,
    8 ants are replayed by the oracle."""
    import torch
    cfg = instances.CONFIGS["c3"]
    xy = instances.make_coords("c3")
    n, k, m = cfg["n"], cfg["k"], cfg["m"]
    col = colony(xy, k=k, m=m, seed=cfg["seed"])
    col.setup()
    col.construct(0)
    col.update_local_best()
    col.update()
    torch.cuda.synchronize()
    lb = _np(col.lbest).copy()
    tau = _np(col.tau).copy()
    col.step_prob = torch.empty((m, n), dtype=torch.float32, device="cuda")
    M = n // 100
    col.construct_partial(1, 1.0, M)
    tours, lengths, slots, probs = (_np(col.tours), _np(col.lengths), _np(col.slots),
                                    _np(col.step_prob))
    say("[partial] c3: checking all tours")
    srt = np.sort(tours, axis=1)
    assert (srt == np.arange(n)).all()
    say("[partial] c3: oracle candidate lists")
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    sample = [0, 1, 255, 511, 512, 700, 1000, 1023]
    tot = check_partial(xy, nn, nnd, tau, cfg["seed"], 1, lb, 1.0, M, tours, lengths, slots,
                        probs, sample, "c3")
    say(f"[partial] c3 sample: {tot}")


def test_partial_rejects_bad_arguments():
    import paper_1709_03187_amd as aco
    xy = instances.make_coords("c1")
    col = colony(xy, k=10, m=4, seed=1)
    col.setup()
    col.construct(0)
    col.update_local_best()
    for p, M in ((1.5, 10), (-0.1, 10), (0.5, 0)):
        with pytest.raises(aco.AcoError) as e:
            col.construct_partial(1, p, M)
        assert e.value.code == aco.ACO_ERR_INVALID_ARG
    saved = col.lbest
    col.lbest = None
    with pytest.raises(aco.AcoError):
        col.construct_partial(1, 0.5, 10)
    col.lbest = saved


def test_partial_with_local_best_pheromone():
    """PartialACO on the P-ACO pheromone (Section 3): after every iteration the
    table is recomputed from the local bests, bit-exactly as the oracle does;
    the next iteration is replayed on it."""
    xy = instances.make_coords("c1")
    k, m, seed, M = 10, 32, 8, 150
    n = len(xy)
    base, delta = 1.0 / (n - 1), 1.0 / m
    col = colony(xy, k=k, m=m, seed=seed, want_prob=True)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    col.construct(0)
    col.update_local_best()
    lbest, lbest_len = _np(col.lbest).copy(), _np(col.lbest_len).copy()
    col.pheromone_from_local_best(base, delta)
    tau, q = orc.pheromone_local_best(nn, lbest, lbest_len, base, delta)
    np.testing.assert_array_equal(_np(col.tau), tau)
    for it in range(1, 5):
        say(f"[partial] local-best pheromone iteration {it}")
        col.construct_partial(it, 0.95, M)
        tours, lengths = _np(col.tours), _np(col.lengths)
        check_partial(xy, nn, nnd, tau, seed, it, lbest, 0.95, M, tours, lengths, _np(col.slots),
                      _np(col.step_prob), range(m), f"pbest it={it}")
        col.update_local_best()
        lbest, lbest_len = orc.update_local_best(lbest, lbest_len, tours, lengths)
        np.testing.assert_array_equal(_np(col.lbest), lbest)
        col.pheromone_from_local_best(base, delta)
        tau, q = orc.pheromone_local_best(nn, lbest, lbest_len, base, delta)
        np.testing.assert_array_equal(_np(col.tau), tau, err_msg=f"it={it}")


@pytest.mark.parametrize("name,M,p", [("c1", 150, 0.95), ("c1", 999, 1.0), ("c1", 1, 1.0),
                                      ("clustered", 40, 0.7)])
def test_kept_length_from_local_best_lengths(name, M, p):
    """The kept part's length taken from the local best's length (minus the
    edges outside the kept part) equals the sum over the kept part; tours are
    replayed by the oracle, lengths compared exactly."""
    import torch
    xy = instances.make_coords("c1") if name == "c1" else \
        instances.clustered_coords(3000, 8, clusters=5, sigma=3e3)
    k, m, seed = 10, 32, 12
    col = colony(xy, k=k, m=m, seed=seed, want_prob=True)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    tau = _np(col.tau).copy()
    col.construct(0)
    col.update_local_best()
    for it in range(1, 4):
        lbest = _np(col.lbest).copy()
        col.construct_ex(it, p_partial=p, max_modify=M, partial=True, use_lbest_len=False)
        ref = (_np(col.tours).copy(), _np(col.lengths).copy(), _np(col.slots).copy())
        col.construct_ex(it, p_partial=p, max_modify=M, partial=True, use_lbest_len=True)
        tours, lengths = _np(col.tours), _np(col.lengths)
        np.testing.assert_array_equal(tours, ref[0])
        np.testing.assert_array_equal(lengths, ref[1])
        np.testing.assert_array_equal(_np(col.slots), ref[2])
        check_partial(xy, nn, nnd, tau, seed, it, lbest, p, M, tours, lengths, _np(col.slots),
                      _np(col.step_prob), range(0, m, 5), f"lbest_len {name} it={it}")
        say(f"[partial] kept length from local best lengths: {name} M={M} it={it}")
        col.update_local_best()
        torch.cuda.synchronize()
