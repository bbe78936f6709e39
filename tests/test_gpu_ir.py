"""GPU parity of the Independent Roulette sampler (Section 3) against the CPU
oracle: full tours, and the paper's combination of PartialACO with
Independent Roulette and pheromone from the local bests.

Choices must equal the oracle's except where the two largest products lie
within 2^-22 of each other (the GPU's weights are the FP64 weights rounded
once to FP32); such steps are counted and kept below 1e-4 of all steps."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import BOUNDARY_RATE, colony, require_gpu, say, threads

pytestmark = pytest.mark.gpu
IR = orc.SAMPLER_INDEPENDENT


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def check_ir(xy, nn, nnd, tau, seed, it, lbest, p, M, tours, lengths, slots, ants, label):
    n, k = nn.shape
    tot = dict(steps=0, near=0)
    for a in ants:
        T = tours[a]
        cnt, oprob = orc.replay_partial(xy, nn, nnd, tau, 1.0, 2.0, seed, it, a, lbest[a], p, M, T,
                                        sampler=IR)
        assert cnt["invalid"] == 0 and cnt["hard_mismatch"] == 0, (label, a, cnt)
        assert cnt["fallback_mismatch"] == 0, (label, a, cnt)
        tot["steps"] += cnt["steps"]
        tot["near"] += cnt["near_boundary_mismatch"]
        keep = cnt["kept"] if cnt["kept"] < n else 1
        assert np.array_equal(np.sort(T), np.arange(n)), (label, a)
        assert lengths[a] == orc.tour_length(xy, T), (label, a)
        sl = slots[a]
        fb = sl[keep:] == 255
        assert np.array_equal(fb, oprob[keep:] < 0), (label, a)
        idx = np.nonzero(~fb)[0] + keep
        assert np.array_equal(nn[T[idx - 1], sl[idx]], T[idx]), (label, a)
    assert tot["near"] <= BOUNDARY_RATE * max(tot["steps"], 1)
    return tot


def test_independent_roulette_full_tours():
    import paper_1709_03187_amd as aco
    xy = instances.make_coords("c1")
    k, m, seed = 10, 32, 6
    col = colony(xy, k=k, m=m, seed=seed)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    tau = _np(col.tau).copy()
    dummy = np.zeros((m, len(xy)), np.int32)
    for it in range(3):
        col.construct_ex(it, sampler=aco.ACO_SAMPLER_INDEPENDENT)
        tours, lengths = _np(col.tours), _np(col.lengths)
        tot = check_ir(xy, nn, nnd, tau, seed, it, dummy, 0.0, 1, tours, lengths, _np(col.slots),
                       range(m), f"ir it={it}")
        say(f"[ir] full it={it}: {tot}")
        col.update()
        tau = orc.update(nn, tau, tours, lengths, 0.1, 32)
        np.testing.assert_array_equal(_np(col.tau), tau)
    # the two samplers differ from the same Philox stream
    col.construct_ex(3, sampler=aco.ACO_SAMPLER_ROULETTE)
    rou = _np(col.tours).copy()
    col.construct_ex(3, sampler=aco.ACO_SAMPLER_INDEPENDENT)
    assert not np.array_equal(rou, _np(col.tours))
    np.testing.assert_array_equal(rou[:, 0], _np(col.tours)[:, 0])


def test_paper_method_partial_independent_local_best_pheromone():
    """PartialACO + Independent Roulette + pheromone from the local bests."""
    import paper_1709_03187_amd as aco
    xy = instances.make_coords("c1")
    k, m, seed, M, p = 10, 32, 9, 100, 0.95
    n = len(xy)
    base, delta = 1.0 / (n - 1), 1.0 / m
    col = colony(xy, k=k, m=m, seed=seed)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    tau = _np(col.tau).copy()
    dummy = np.zeros((m, n), np.int32)
    col.construct_ex(0, sampler=aco.ACO_SAMPLER_INDEPENDENT)
    tours, lengths = _np(col.tours), _np(col.lengths)
    check_ir(xy, nn, nnd, tau, seed, 0, dummy, 0.0, 1, tours, lengths, _np(col.slots), range(m),
             "paper it=0")
    col.update_local_best()
    lbest, lbest_len = orc.update_local_best(dummy, np.full(m, 2**63 - 1), tours, lengths)
    col.pheromone_from_local_best(base, delta)
    tau, _ = orc.pheromone_local_best(nn, lbest, lbest_len, base, delta)
    np.testing.assert_array_equal(_np(col.tau), tau)
    for it in range(1, 5):
        col.construct_ex(it, sampler=aco.ACO_SAMPLER_INDEPENDENT, p_partial=p, max_modify=M,
                         partial=True)
        tours, lengths = _np(col.tours), _np(col.lengths)
        tot = check_ir(xy, nn, nnd, tau, seed, it, lbest, p, M, tours, lengths, _np(col.slots),
                       range(m), f"paper it={it}")
        say(f"[ir] paper method it={it}: {tot}")
        col.update_local_best()
        lbest, lbest_len = orc.update_local_best(lbest, lbest_len, tours, lengths)
        np.testing.assert_array_equal(_np(col.lbest), lbest)
        col.pheromone_from_local_best(base, delta)
        tau, _ = orc.pheromone_local_best(nn, lbest, lbest_len, base, delta)
        np.testing.assert_array_equal(_np(col.tau), tau)



@pytest.mark.parametrize("n,k", [(300, 20), (257, 33), (401, 64), (150, 7)])
def test_independent_roulette_wide_and_narrow_rows(n, k):
    """Rows of 7 to 64 candidates (scan widths 8, 32 and 64; 2 to 16 Philox
    blocks of uniforms per step staged in LDS), full and partial tours."""
    import paper_1709_03187_amd as aco
    xy = instances.uniform_coords(n, 40 + k)
    m, seed, M, p = 8, 17, n // 3, 1.0
    col = colony(xy, k=k, m=m, seed=seed)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    tau = _np(col.tau).copy()
    dummy = np.zeros((m, n), np.int32)
    col.construct_ex(0, sampler=aco.ACO_SAMPLER_INDEPENDENT)
    tours, lengths = _np(col.tours), _np(col.lengths)
    tot = check_ir(xy, nn, nnd, tau, seed, 0, dummy, 0.0, 1, tours, lengths, _np(col.slots),
                   range(m), f"ir n={n} k={k}")
    col.update_local_best()
    lbest, _ = orc.update_local_best(dummy, np.full(m, 2**63 - 1), tours, lengths)
    col.construct_ex(1, sampler=aco.ACO_SAMPLER_INDEPENDENT, p_partial=p, max_modify=M,
                     partial=True)
    tot2 = check_ir(xy, nn, nnd, tau, seed, 1, lbest, p, M, _np(col.tours), _np(col.lengths),
                    _np(col.slots), range(m), f"ir partial n={n} k={k}")
    say(f"[ir] n={n} k={k}: full {tot}, partial {tot2}")

def test_independent_roulette_full_size_sample():
    import paper_1709_03187_amd as aco
    cfg = instances.CONFIGS["c3"]
    xy = instances.make_coords("c3")
    n, k, m = cfg["n"], cfg["k"], cfg["m"]
    col = colony(xy, k=k, m=m, seed=cfg["seed"])
    col.setup()
    tau = _np(col.tau).copy()
    col.construct_ex(0, sampler=aco.ACO_SAMPLER_INDEPENDENT)
    tours, lengths, slots = _np(col.tours), _np(col.lengths), _np(col.slots)
    say("[ir] c3: every tour a permutation")
    assert (np.sort(tours, axis=1) == np.arange(n)).all()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    tot = check_ir(xy, nn, nnd, tau, cfg["seed"], 0, np.zeros((m, n), np.int32), 0.0, 1, tours,
                   lengths, slots, [0, 100, 511, 1023], "c3 ir")
    say(f"[ir] c3 sample: {tot}")


def test_independent_roulette_rejects_step_probabilities():
    import torch
    import paper_1709_03187_amd as aco
    xy = instances.make_coords("c1")
    col = colony(xy, k=10, m=4, seed=1, want_prob=True)
    col.setup()
    with pytest.raises(aco.AcoError) as e:
        aco.aco_construct_ex(col.xy, col.n, col.k, col.nn, col.nnd, col.eta_b, col.grid, col.tau,
                             4, 0, 1.0, 1, 0, aco.ACO_SAMPLER_INDEPENDENT, 0.0, 1, None, col.tours,
                             col.lengths, col.slots, col.step_prob, col.cws)
    assert e.value.code == aco.ACO_ERR_INVALID_ARG
    with pytest.raises(aco.AcoError):
        col.construct_ex(0, sampler=7)
    torch.cuda.synchronize()
