"""GPU parity of the batched colonies (thousands of independent instances in
one persistent launch) against the CPU oracle run instance by instance.

The oracle has no notion of a batch: every instance is the single-instance
method with its own cities numbered from 0 and ants 0..m-1."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import check_tours, require_gpu, say, threads

pytestmark = pytest.mark.gpu

K, M, SEED = 12, 64, 4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def make_batch(count, iterations=3, k=K, m=M, seed=SEED, extra=()):
    import paper_1709_03187_amd as aco
    xy, off, sizes = instances.make_batched("c4", count=count)
    if extra:
        parts = [xy] + [np.asarray(e, np.int32) for e in extra]
        xy = np.concatenate(parts)
        sizes = np.concatenate([sizes, [len(e) for e in extra]])
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bt = aco.Batch(xy, off, k=k, m=m, seed=seed, iterations=iterations)
    return bt, xy, off, sizes


def state(bt):
    import torch
    torch.cuda.synchronize()
    N, B, k, m = bt.N, bt.B, bt.params.k, bt.params.m
    return dict(
        nn=bt.view("nn", torch.int32, N * k).cpu().numpy().reshape(N, k),
        nnd=bt.view("nnd", torch.int32, N * k).cpu().numpy().reshape(N, k),
        rev=bt.view("rev", torch.int8, N * k).cpu().numpy().reshape(N, k),
        eta_b=bt.view("eta_b", torch.float32, N * k).cpu().numpy().reshape(N, k),
        tau=bt.view("tau", torch.float32, N * k).cpu().numpy().reshape(N, k),
        tours=bt.view("tours", torch.int32, N * m).cpu().numpy(),
        slots=bt.view("slots", torch.uint8, N * m).cpu().numpy(),
        lengths=bt.view("lengths", torch.int64, B * m).cpu().numpy().reshape(B, m),
        best_tours=bt.best_tours.cpu().numpy(),
        best_lens=bt.best_lens.cpu().numpy(),
    )


def inst(S, off, b, m=M):
    lo, hi = int(off[b]), int(off[b + 1])
    n = hi - lo
    k = S["nn"].shape[1]
    return dict(n=n, k=k, nn=S["nn"][lo:hi], nnd=S["nnd"][lo:hi], rev=S["rev"][lo:hi],
                eta_b=S["eta_b"][lo:hi], tau=S["tau"][lo:hi],
                tours=S["tours"][m * lo:m * hi].reshape(m, n),
                slots=S["slots"][m * lo:m * hi].reshape(m, n),
                lengths=S["lengths"][b], best_tour=S["best_tours"][lo:hi],
                best_len=int(S["best_lens"][b]))


@pytest.mark.parametrize("layout", [1, 3])
def test_batch_setup_and_iterations_match_oracle(layout):
    """layout 1: one ant per wave; 3: four ants per wave (one per 16-lane row)."""
    # 20 instances of the batched workload plus the smallest legal size (n = k + 1)
    tiny = instances.uniform_coords(K + 1, 99)
    bt, xy, off, sizes = make_batch(20, extra=[tiny])
    replay_batch(bt, xy, off, K, 3, layout)


def replay_batch(bt, xy, off, K, iterations, layout):
    """Set-up checked against the oracle per instance, then `iterations`
    iterations one launch at a time, every ant of every instance replayed and
    the pheromone and bests compared after each."""
    import torch
    say(f"[batch] setup B={bt.B} N={bt.N} k={K}")
    bt.setup()
    S = state(bt)
    ref = {}
    for b in range(bt.B):
        xb = xy[off[b]:off[b + 1]]
        I = inst(S, off, b)
        nn, nnd = orc.knn_rows(xb, K, threads=threads())
        np.testing.assert_array_equal(I["nn"], nn)
        np.testing.assert_array_equal(I["nnd"], nnd)
        np.testing.assert_array_equal(I["rev"], orc.rev(nn))
        eta = 1.0 / np.maximum(nnd, 1).astype(np.float64)
        np.testing.assert_allclose(I["eta_b"], (eta * eta).astype(np.float32), rtol=1.2e-7)
        tour, L = orc.nn_tour(xb, nn, nnd)
        np.testing.assert_array_equal(I["best_tour"], tour)
        assert I["best_len"] == L
        tau = np.full((I["n"], I["k"]), orc.tau0(I["n"], L), np.float32)
        np.testing.assert_array_equal(I["tau"], tau)
        ref[b] = dict(xy=xb, nn=nn, nnd=nnd, tau=tau, best=L)
    steps = near = 0
    for t in range(iterations):
        say(f"[batch] iteration {t}")
        ib = torch.empty((bt.B, 1), dtype=torch.int64, device="cuda")
        # one ant per wave also records the step probabilities
        prob = torch.empty(bt.N * M, dtype=torch.float32, device="cuda") if layout != 3 else None
        bt.iterate(t, 1, waves=8, layout=layout, iter_best=ib, step_prob=prob)
        S = state(bt)
        P = None if prob is None else prob.cpu().numpy()
        ibn = ib.cpu().numpy()[:, 0]
        for b in range(bt.B):
            I, R = inst(S, off, b), ref[b]
            pb = None if P is None else P[M * off[b]:M * off[b + 1]].reshape(M, I["n"])
            tot = check_tours(R["xy"], R["nn"], R["nnd"], R["tau"], 1.0, 2.0, SEED, t,
                              I["tours"], I["lengths"], I["slots"], pb, np.arange(M),
                              label=f"batch b={b} t={t}")
            steps += tot["steps"]
            near += tot["near_boundary_mismatch"]
            assert ibn[b] == I["lengths"].min()
            R["best"] = min(R["best"], int(I["lengths"].min()))
            assert I["best_len"] == R["best"]
            assert orc.tour_length(R["xy"], I["best_tour"]) == R["best"]
            R["tau"] = orc.update(R["nn"], R["tau"], I["tours"], I["lengths"], 0.1, 32)
            np.testing.assert_array_equal(I["tau"], R["tau"], err_msg=f"b={b} t={t}")
    assert near <= 1e-4 * steps
    return S


CONFIGS = [(1, 1, 4), (2, 1, 4), (4, 1, 4), (8, 1, 4), (16, 1, 4), (4, 2, 4), (8, 2, 4),
           (16, 2, 4), (4, 1, 8), (16, 1, 8), (8, 2, 8), (1, 3, 4), (4, 3, 4), (16, 3, 4),
           (2, 3, 8), (8, 3, 8), (16, 3, 8)]


def test_batch_invariance_across_configurations():
    import torch
    results = []
    for waves, layout, occ in CONFIGS:
        say(f"[batch] config waves={waves} layout={layout} occupancy={occ}")
        bt, xy, off, sizes = make_batch(48)
        bt.setup()
        ib = torch.empty((bt.B, 3), dtype=torch.int64, device="cuda")
        bt.iterate(0, 3, waves=waves, layout=layout, iter_best=ib, occupancy=occ)
        S = state(bt)
        results.append((S["tau"], S["best_lens"], S["best_tours"], ib.cpu().numpy()))
    for r in results[1:]:
        for a, b in zip(results[0], r):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("m,k", [(10, 12), (7, 8), (13, 16)])
def test_batch_four_ants_per_wave_partial_groups(m, k):
    """Ant counts that leave some of a wave's four rows empty, and k = 8, 12, 16:
    four ants per wave give the same state as one ant per wave."""
    import torch
    results = []
    for waves, layout in ((4, 1), (4, 3), (2, 3), (1, 3)):
        bt, xy, off, sizes = make_batch(12, k=k, m=m)
        bt.setup()
        ib = torch.empty((bt.B, 3), dtype=torch.int64, device="cuda")
        bt.iterate(0, 3, waves=waves, layout=layout, iter_best=ib, occupancy=4)
        S = state(bt)
        results.append((S["tau"], S["best_lens"], S["best_tours"], S["tours"], S["slots"],
                        S["lengths"], ib.cpu().numpy()))
    for r in results[1:]:
        for a, b in zip(results[0], r):
            np.testing.assert_array_equal(a, b)


def test_batch_four_ants_rejects_wide_rows():
    import paper_1709_03187_amd as aco
    bt, xy, off, sizes = make_batch(4, k=20, m=8)
    bt.setup()
    with pytest.raises(aco.AcoError) as e:
        bt.iterate(0, 1, waves=4, layout=aco.ACO_VIS_BITS_X4)
    assert e.value.code == aco.ACO_ERR_INVALID_ARG


def test_batch_k_auto_run_equals_oracle_replayed_fixed_k():
    """k = 0: the library picks k from 8, 10, 12, 16 by time to equal quality;
    the run then equals a fixed-k run of the chosen k that the oracle replays
    iteration by iteration."""
    import torch
    bt, xy, off, sizes = make_batch(12, iterations=3, k=0)
    ib = torch.empty((bt.B, 3), dtype=torch.int64, device="cuda")
    tuned = bt.run(autotune=0, iter_best=ib)
    k = tuned[3]
    say(f"[batch] k-auto chose k={k}")
    assert k in (8, 10, 12, 16) and bt.params.k == k
    A = state(bt)
    ref, *_ = make_batch(12, iterations=3, k=k)
    Bst = replay_batch(ref, xy, off, k, 3, 1)
    for f in ("tau", "tours", "slots", "lengths", "best_tours", "best_lens"):
        np.testing.assert_array_equal(A[f], Bst[f], err_msg=f)


def test_batch_autotuned_run_equals_fixed_configuration():
    """Every candidate shape is timed on iteration 0 from the restored set-up
    state; the run in the chosen shape equals a fixed one in every iteration."""
    import torch
    bt, xy, off, sizes = make_batch(40, iterations=9)
    ib = torch.empty((bt.B, 9), dtype=torch.int64, device="cuda")
    tuned = bt.run(autotune=1, iter_best=ib)
    assert tuned[0] in (4, 8, 16) and tuned[1] in (1, 2, 3) and tuned[2] in (4, 8)
    assert tuned[3] == K
    A = state(bt)
    bt2, *_ = make_batch(40, iterations=9)
    bt2.setup()
    ib2 = torch.empty((bt2.B, 9), dtype=torch.int64, device="cuda")
    bt2.iterate(0, 9, waves=4, layout=1, iter_best=ib2)
    Bst = state(bt2)
    np.testing.assert_array_equal(A["tau"], Bst["tau"])
    np.testing.assert_array_equal(A["best_lens"], Bst["best_lens"])
    np.testing.assert_array_equal(A["best_tours"], Bst["best_tours"])
    np.testing.assert_array_equal(ib.cpu().numpy(), ib2.cpu().numpy())


def test_batch_graph_capture_and_replay():
    """The iterate launch captured in a HIP graph: every replay equals the
    eager call it stands for (with eager work and synchronisation between)."""
    import torch
    eager, xy, off, sizes = make_batch(32)
    eager.setup()
    graphed, *_ = make_batch(32)
    graphed.setup()
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        graphed.iterate(0, 2, waves=8, layout=1)
    for rep in range(3):
        eager.iterate(0, 2, waves=8, layout=1)
        g.replay()
        junk = torch.ones(1 << 20, device="cuda").sum()   # unrelated eager work in between
        torch.cuda.synchronize()
        A, Bst = state(eager), state(graphed)
        for key in ("tau", "best_lens", "best_tours", "lengths"):
            np.testing.assert_array_equal(A[key], Bst[key], err_msg=f"replay {rep} {key}")
        assert float(junk.item()) == float(1 << 20)


def test_batch_full_size_sample():
    """All 4,096 instances of the batched workload, one iteration; a sample of
    instances is replayed and updated by the oracle, every tour is checked."""
    import torch
    cfg = instances.CONFIGS["c4"]
    bt, xy, off, sizes = make_batch(cfg["instances"], iterations=1)
    say(f"[batch] full set-up B={bt.B} N={bt.N}")
    bt.setup()
    tau_before = bt.view("tau", torch.float32, bt.N * K).cpu().numpy().reshape(bt.N, K).copy()
    ib = torch.empty((bt.B, 1), dtype=torch.int64, device="cuda")
    bt.iterate(0, 1, iter_best=ib)
    S = state(bt)
    ibn = ib.cpu().numpy()[:, 0]
    order = np.argsort(-sizes, kind="stable")
    sample = sorted(set([int(order[0]), int(order[1]), int(order[-1]), 0, 1, 2047, 4095]))
    for b in range(bt.B):
        I = inst(S, off, b)
        n = I["n"]
        assert np.array_equal(np.sort(I["tours"], axis=1), np.broadcast_to(np.arange(n), (M, n)))
        assert ibn[b] == I["lengths"].min()
    for b in sample:
        say(f"[batch] full-size replay of instance {b} (n={sizes[b]})")
        xb = xy[off[b]:off[b + 1]]
        I = inst(S, off, b)
        nn, nnd = orc.knn_rows(xb, K, threads=threads())
        np.testing.assert_array_equal(I["nn"], nn)
        tau = tau_before[off[b]:off[b + 1]]
        check_tours(xb, nn, nnd, tau, 1.0, 2.0, SEED, 0, I["tours"], I["lengths"], I["slots"],
                    None, np.arange(M), label=f"full b={b}")
        np.testing.assert_array_equal(I["tau"], orc.update(nn, tau, I["tours"], I["lengths"],
                                                           0.1, 32))


def test_batch_rejects_bad_input():
    import paper_1709_03187_amd as aco
    xy, off, sizes = instances.make_batched("c4", count=4)
    bad = np.array([0, 5, 5 + sizes[1]], np.int64)   # second instance too small for k = 12
    with pytest.raises(aco.AcoError) as e:
        aco.Batch(xy[:bad[-1]], bad, k=K, m=M).setup()
    assert e.value.code == aco.ACO_ERR_INVALID_ARG
    same = np.concatenate([xy[:sizes[0]], np.full((20, 2), 7, np.int32)])
    off2 = np.array([0, sizes[0], sizes[0] + 20], np.int64)
    with pytest.raises(aco.AcoError) as e:
        aco.Batch(same, off2, k=K, m=M).setup()
    assert e.value.code == aco.ACO_ERR_DEGENERATE
