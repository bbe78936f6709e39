"""GPU parity: candidate lists, NN-tour initialisation, tour construction and
pheromone update of the HIP path against the CPU oracle, on the small
workloads (n = 1,000 uniform; n = 20,000 uniform) and edge cases."""
import numpy as np
import pytest

import oracle as orc
from oracle import exact
from paper_1709_03187_amd import instances
from tests.gpu_util import check_tours, colony, require_gpu, say, threads, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def edge_instances():
    line = np.stack([np.arange(300) * 7 % 1000, np.zeros(300)], 1).astype(np.int32)
    ties = instances.uniform_coords(500, 17, hi=30)            # many equal distances, duplicates
    clus = instances.clustered_coords(3000, 8, clusters=5, sigma=3e3)
    tiny = instances.uniform_coords(3, 2)
    k64 = instances.uniform_coords(65, 3)
    neg = instances.uniform_coords(400, 4, hi=2 * 10**8) - 10**8
    # rows that are not a power of two wide: scan widths 8, 32 and 64
    k7 = instances.uniform_coords(333, 5)
    k20 = instances.uniform_coords(517, 6)
    k33 = instances.uniform_coords(301, 7)
    return {"line": (line, 6), "ties": (ties, 12), "clustered": (clus, 16), "n3": (tiny, 2),
            "k64": (k64, 64), "negative": (neg, 10), "k7": (k7, 7), "k20": (k20, 20),
            "k33": (k33, 33)}


CASES = {"c1": (instances.make_coords("c1"), 10), **edge_instances()}


@pytest.mark.parametrize("name", list(CASES))
def test_candidates_and_nn_tour(name):
    xy, k = CASES[name]
    n = len(xy)
    say(f"[candidates] {name} n={n} k={k}")
    col = colony(xy, k=k, m=4)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    np.testing.assert_array_equal(to_np(col.nnd), nnd)
    np.testing.assert_array_equal(to_np(col.nn), nn)
    np.testing.assert_array_equal(to_np(col.rev), orc.rev(nn))
    eta = 1.0 / np.maximum(nnd, 1).astype(np.float64)
    np.testing.assert_allclose(to_np(col.eta_b), (eta * eta).astype(np.float32), rtol=1.2e-7)
    tour, L = orc.nn_tour(xy, nn, nnd)
    np.testing.assert_array_equal(to_np(col.nn_tour), tour)
    assert col.L_nn == L
    assert np.float32(col.tau0) == orc.tau0(n, L)
    assert np.all(to_np(col.tau) == orc.tau0(n, L))


def test_candidates_c2():
    xy = instances.make_coords("c2")
    say("[candidates] c2")
    col = colony(xy, k=16, m=4)
    col.setup()
    nn, nnd = orc.knn_rows(xy, 16, threads=threads())
    np.testing.assert_array_equal(to_np(col.nn), nn)
    np.testing.assert_array_equal(to_np(col.nnd), nnd)
    tour, L = orc.nn_tour(xy, nn, nnd)
    np.testing.assert_array_equal(to_np(col.nn_tour), tour)
    assert col.L_nn == L


def run_and_check(xy, k, m, alpha, beta, rho, iterations, seed, shift=32, tau_noise=False,
                  label="", report=None):
    """Iterate on the GPU; every iteration replay all ants with the oracle and
    check the pheromone bit-exactly against the oracle's update."""
    import torch
    n = len(xy)
    col = colony(xy, k=k, m=m, alpha=alpha, beta=beta, rho=rho, seed=seed, deposit_shift=shift,
                 want_prob=True)
    col.setup()
    nn, nnd = orc.knn_rows(xy, k, threads=threads())
    L_nn = orc.nn_tour(xy, nn, nnd)[1]
    tau = np.full((n, k), orc.tau0(n, L_nn), np.float32)
    if tau_noise:   # non-uniform pheromone exercises the roulette
        rng = np.random.default_rng(seed)
        tau = (tau * rng.uniform(0.05, 20.0, size=tau.shape)).astype(np.float32)
        col.tau.copy_(torch.from_numpy(tau))
    np.testing.assert_array_equal(to_np(col.tau), tau)
    steps = 0
    totals = {}
    for it in range(iterations):
        say(f"[run] {label} iteration {it}")
        col.construct(it)
        torch.cuda.synchronize()
        tours, lengths, slots = to_np(col.tours), to_np(col.lengths), to_np(col.slots)
        probs = to_np(col.step_prob)
        tot = check_tours(xy, nn, nnd, tau, alpha, beta, seed, it, tours, lengths, slots, probs,
                          np.arange(m), label=f"{label} it {it}")
        for f, v in tot.items():
            totals[f] = totals.get(f, 0) + v
        steps += tot["steps"]
        col.update()
        torch.cuda.synchronize()
        tau = orc.update(nn, tau, tours, [orc.tour_length(xy, t) for t in tours], rho, shift)
        np.testing.assert_array_equal(to_np(col.tau), tau, err_msg=f"{label} it {it} tau")
        if report:
            report(f"\n[{label}] iteration {it}: oracle replayed all {m} ants, {tot}; "
                   f"pheromone bit-exact")
    say(f"[run] {label} totals {totals}")
    return totals


def test_c1_full_run():
    cfg = instances.CONFIGS["c1"]
    run_and_check(instances.make_coords("c1"), cfg["k"], cfg["m"], cfg["alpha"], cfg["beta"],
                  cfg["rho"], cfg["iterations"], cfg["seed"], label="c1")


@pytest.mark.parametrize("alpha,beta,rho,shift", [(1.0, 2.0, 0.5, 40), (0.0, 0.0, 0.1, 32),
                                                  (2.5, 3.0, 1.0, 32), (1.0, 5.0, 0.02, 62),
                                                  (1.0, 2.0, 0.3, 0)])
def test_parameter_variants(alpha, beta, rho, shift):
    xy = instances.uniform_coords(700, 21)
    run_and_check(xy, 8, 16, alpha, beta, rho, 3, 99, shift=shift, tau_noise=True,
                  label=f"a{alpha} b{beta} r{rho} s{shift}")


@pytest.mark.parametrize("name", ["ties", "clustered", "line", "n3", "k64", "negative", "k7",
                                  "k20", "k33"])
def test_edge_cases_run(name):
    xy, k = CASES[name]
    run_and_check(xy, k, 8, 1.0, 2.0, 0.1, 2, 5, tau_noise=True, label=name)


def test_c2_iterations(report):
    cfg = instances.CONFIGS["c2"]
    xy = instances.make_coords("c2")
    tot = run_and_check(xy, cfg["k"], cfg["m"], cfg["alpha"], cfg["beta"], cfg["rho"], 5,
                        cfg["seed"], label="c2", report=report)
    assert tot["near_boundary_mismatch"] <= 1e-4 * tot["steps"]


def test_update_without_slots_and_custom_tours():
    import torch
    # tours around a circle: every edge, the closing one included, is a candidate edge
    n, k, m = 64, 4, 5
    ang = 2 * np.pi * np.arange(n) / n
    xy = np.stack([np.rint(1e5 * np.cos(ang)), np.rint(1e5 * np.sin(ang))], 1).astype(np.int32)
    col = colony(xy, k=k, m=m)
    col.setup()
    nn, _ = orc.knn_rows(xy, k)
    rng = np.random.default_rng(0)
    tours = np.stack([np.roll(np.arange(n), -s) for s in range(m)]).astype(np.int32)
    tours[1] = tours[1][::-1]
    tours[4] = rng.permutation(n)
    lengths = np.array([orc.tour_length(xy, t) for t in tours], np.int64)
    col.tours.copy_(torch.from_numpy(tours))
    col.lengths.copy_(torch.from_numpy(lengths))
    tau = to_np(col.tau)
    col.update(use_slots=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(col.tau), orc.update(nn, tau, tours, lengths, 0.1, 32))


def test_best_tracking():
    import torch
    xy = instances.uniform_coords(900, 6)
    col = colony(xy, k=10, m=24)
    col.setup()
    iter_best = torch.empty(6, dtype=torch.int64, device="cuda")
    lens = []
    for it in range(6):
        col.construct(it)
        col.track_best(iter_best[it:it + 1])
        lens.append(to_np(col.lengths).copy())
        col.update()
    torch.cuda.synchronize()
    ib = to_np(iter_best)
    np.testing.assert_array_equal(ib, [L.min() for L in lens])
    best = min(col.L_nn, int(ib.min()))
    assert int(to_np(col.best_len)[0]) == best
    bt = to_np(col.best_tour)
    assert np.array_equal(np.sort(bt), np.arange(900))
    assert orc.tour_length(xy, bt) == best


def test_aco_run_matches_stepwise_and_oracle():
    import torch
    import paper_1709_03187_amd as aco
    cfg = instances.CONFIGS["c1"]
    xy = instances.make_coords("c1")
    n, k, m, iters = len(xy), cfg["k"], cfg["m"], cfg["iterations"]
    p = aco.AcoParams(m=m, k=k, alpha=cfg["alpha"], beta=cfg["beta"], rho=cfg["rho"],
                      iterations=iters, deposit_shift=32, seed=cfg["seed"])
    ws = torch.empty(aco.aco_run_workspace_bytes(n, p), dtype=torch.uint8, device="cuda")
    xy_d = torch.from_numpy(xy).cuda()
    best_tour = torch.empty(n, dtype=torch.int32, device="cuda")
    best_len = torch.empty(1, dtype=torch.int64, device="cuda")
    iter_best = torch.empty(iters, dtype=torch.int64, device="cuda")
    tau_out = torch.empty((n, k), dtype=torch.float32, device="cuda")
    say("[aco_run] c1")
    aco.aco_run(xy_d, n, p, best_tour, best_len, iter_best, tau_out, ws)
    torch.cuda.synchronize()
    ref = orc.run(xy, m, k, cfg["alpha"], cfg["beta"], cfg["rho"], iters, cfg["seed"],
                  threads=threads())
    # with no near-boundary draw on the way the two trajectories are identical
    np.testing.assert_array_equal(to_np(iter_best), ref["iter_best"])
    np.testing.assert_array_equal(to_np(tau_out), ref["tau"])
    assert int(to_np(best_len)[0]) == ref["best_len"]
    np.testing.assert_array_equal(to_np(best_tour), ref["best_tour"])


def test_aco_run_with_learned_heuristic_equals_stepwise_colony():
    """eta_mode = ACO_ETA_LEARNED: aco_run scores the candidate edges with the
    network and runs the loop on sigmoid(z)^beta; the same calls made one by
    one (features, forward, then the loop) give bit-identical results."""
    import torch
    import paper_1709_03187_amd as aco
    xy = instances.uniform_coords(1500, 41)
    n, k, m, iters, beta = len(xy), 12, 32, 5, 6.0
    theta = torch.from_numpy(instances.mlp_parameters(3)).cuda()
    p = aco.AcoParams(m=m, k=k, alpha=1.0, beta=beta, rho=0.1, iterations=iters,
                      deposit_shift=32, seed=8, eta_mode=aco.ACO_ETA_LEARNED,
                      mlp_w=theta.data_ptr())
    ws = torch.empty(aco.aco_run_workspace_bytes(n, p), dtype=torch.uint8, device="cuda")
    xy_d = torch.from_numpy(xy).cuda()
    best_tour = torch.empty(n, dtype=torch.int32, device="cuda")
    best_len = torch.empty(1, dtype=torch.int64, device="cuda")
    iter_best = torch.empty(iters, dtype=torch.int64, device="cuda")
    tau_out = torch.empty((n, k), dtype=torch.float32, device="cuda")
    aco.aco_run(xy_d, n, p, best_tour, best_len, iter_best, tau_out, ws)
    col = colony(xy, k=k, m=m, beta=beta, seed=8, theta=theta)
    col.setup()
    ib = torch.empty(iters, dtype=torch.int64, device="cuda")
    for it in range(iters):
        col.iterate(it, ib[it:it + 1])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(iter_best), to_np(ib))
    np.testing.assert_array_equal(to_np(tau_out), to_np(col.tau))
    assert int(best_len.item()) == int(col.best_len.item())
    np.testing.assert_array_equal(to_np(best_tour), to_np(col.best_tour))
    # and the table really is the network's, not 1/d
    eta = 1.0 / np.maximum(to_np(col.nnd), 1).astype(np.float64)
    assert not np.array_equal(to_np(col.eta_b), (eta ** beta).astype(np.float32))


def test_ant_split_and_determinism():
    import torch
    xy = instances.uniform_coords(1500, 8)
    col = colony(xy, k=12, m=20)
    col.setup()
    col.construct(3)
    torch.cuda.synchronize()
    a = to_np(col.tours).copy()
    col.construct(3, m=7, ant0=0)
    torch.cuda.synchronize()
    b1 = to_np(col.tours)[:7].copy()
    # ants 7..19 written to the first rows of the buffers
    col.construct(3, m=13, ant0=7)
    torch.cuda.synchronize()
    b2 = to_np(col.tours)[:13].copy()
    np.testing.assert_array_equal(a[:7], b1)
    np.testing.assert_array_equal(a[7:], b2)


def test_one_and_four_ants_per_workgroup_agree():
    """More ants than four per CU run one per workgroup; the same ants launched
    four per workgroup draw the same tours."""
    import torch
    xy = instances.uniform_coords(300, 9)
    m = 1100
    col = colony(xy, k=8, m=m)
    col.setup()
    col.construct(2)
    torch.cuda.synchronize()
    many = to_np(col.tours).copy()
    assert (np.sort(many, axis=1) == np.arange(300)).all()
    col.construct(2, m=97, ant0=1003)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(col.tours)[:97], many[1003:1100])
    col.construct(2, m=5, ant0=0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(col.tours)[:5], many[:5])


def test_sampling_distribution_tiny():
    """GPU tour frequencies on a 5-city instance against the exact distribution."""
    import math
    import torch
    n, k = 5, 4
    xy = instances.uniform_coords(n, 45, hi=1000)
    pts = [tuple(map(int, p)) for p in xy]
    col = colony(xy, k=k, m=50_000)
    col.setup()
    rng = np.random.default_rng(3)
    tau = rng.uniform(1e-6, 1e-3, size=(n, k)).astype(np.float32)
    col.tau.copy_(torch.from_numpy(tau))
    col.construct(0)
    torch.cuda.synchronize()
    nn, nnd = exact.candidate_lists(pts, k)
    probs = {}
    for s in range(n):
        ps = exact.start_probability(s, n)
        for t, p in exact.tour_distribution(pts, nn, nnd, tau.tolist(), s).items():
            probs[t] = ps * p
    counts = {}
    for t in map(tuple, to_np(col.tours).tolist()):
        counts[t] = counts.get(t, 0) + 1
    assert set(counts) <= set(probs)
    stat, dof = 0.0, -1
    for key, p in probs.items():
        e = float(p) * 50_000
        stat += (counts.get(key, 0) - e) ** 2 / e
        dof += 1
    z = 4.26
    crit = dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3
    assert stat < crit, (stat, dof)


def test_invalid_arguments_leave_outputs_untouched():
    import torch
    import paper_1709_03187_amd as aco
    xy = instances.uniform_coords(100, 1)
    col = colony(xy, k=8, m=4)
    col.setup()
    col.tours.fill_(-7)
    with pytest.raises(aco.AcoError) as e:
        aco.aco_construct_tours(col.xy, 100, 8, col.nn, col.nnd, col.eta_b, col.grid, col.tau,
                                4, 0, -1.0, 1, 0, col.tours, col.lengths, col.slots, None,
                                col.cws)
    assert e.value.code == aco.ACO_ERR_INVALID_ARG
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(aco.AcoError) as e:
        aco.aco_construct_tours(col.xy, 100, 8, col.nn, col.nnd, col.eta_b, col.grid, col.tau,
                                4, 0, 1.0, 1, 0, col.tours, col.lengths, col.slots, None, small)
    assert e.value.code == aco.ACO_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert (col.tours == -7).all()
    same = np.zeros((10, 2), np.int32) + 5
    with pytest.raises(aco.AcoError) as e:
        colony(same, k=3, m=2).setup()
    assert e.value.code == aco.ACO_ERR_DEGENERATE
    big = instances.uniform_coords(10, 1)
    big[3, 0] = aco.ACO_COORD_LIMIT + 1
    with pytest.raises(aco.AcoError) as e:
        colony(big, k=3, m=2).setup()
    assert e.value.code == aco.ACO_ERR_INVALID_ARG
