"""Benchmark of the ACO hot path on one MI355X.

Workload: n = 200,000 clustered cities (100 Gaussian clusters, sigma = 1e4,
integer coordinates), m = 1,024 ants, k = 16 candidates, alpha = 1, beta = 2,
rho = 0.1, Philox seed 3.  A step is one ACO iteration: tour construction of
all ants, best tracking, and the pheromone update.  Candidate lists, grid and
NN-tour initialisation run once before the timed region.

Prints one JSON line.  `value` = ant-steps per second over whole iterations,
m * (n - 1) ant-steps per iteration.  `roofline` prices the construction
kernel by its algorithmic bytes per ant-step.  `cpu_baseline` times the CPU
oracle (threads over ants) on a fixed sample of ants of the same workload.
`equal_time_c1` and `equal_time_c2` run the GPU and the oracle to
completion on n = 1,000 and n = 20,000 and compare their bests at the GPU's
wall time and at equal iterations.
Further objects report the batched colonies (4,096 instances, one
persistent launch, autotuned), the learned heuristic (training on the GPU,
kernel rates, and the equal-wall-clock comparison with plain eta) and
PartialACO (rebuilding at most 1% of each ant's local best per iteration,
run for the plain colony's wall time), Independent Roulette, and windowed
2-opt (alone on constructed tours, and inside PartialACO with p = 0.001,
W = 500).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-batched] [--no-learned] [--no-partial]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "c3"


def construct_bytes_per_step(k: int) -> int:
    """Algorithmic bytes of one ant-step of construction: the candidate row
    {city int32, weight fp32} x k, the tour entry (int32), the slot record
    (uint8) and the chosen edge's distance (int32)."""
    return 8 * k + 4 + 1 + 4


def construct_bytes_per_launch(n: int, m: int, k: int) -> int:
    """Algorithmic bytes of one aco_construct_tours call: m (n - 1) ant-steps,
    plus the choice-weight pass over the n x k table (read tau, eta^beta and
    the candidate index, 12 bytes; write the packed {city, weight}, 8 bytes)."""
    return m * (n - 1) * construct_bytes_per_step(k) + 20 * n * k


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_construct_c3_n200k_m1024_k16.md")
TRAFFIC_SOURCES = ["paper_1709_03187_amd/csrc/construct.hip",
                   "paper_1709_03187_amd/csrc/colony.hpp",
                   "paper_1709_03187_amd/csrc/device.hpp",
                   "paper_1709_03187_amd/csrc/common.hpp"]
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batched_c4_4096inst_m64_k12.md")
BATCH_TRAFFIC_SOURCES = ["paper_1709_03187_amd/csrc/batch.hip",
                         "paper_1709_03187_amd/csrc/colony.hpp",
                         "paper_1709_03187_amd/csrc/colony_x4.hpp",
                         "paper_1709_03187_amd/csrc/device.hpp",
                         "paper_1709_03187_amd/csrc/common.hpp"]
# Random 64-bit atomic adds per second on one MI355X (a probe of 2^27 hashed
# adds from 8,192 workgroups; the same from 1 MiB to 256 MiB buffers).
ATOMIC_RATE_PROBE = 23.7e9


def counter_summary(path, sources):
    """Fields of a committed counter summary, or None when the sources it was
    taken from changed since (hash mismatch) or it is missing."""
    import hashlib
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if ": " in line and not line.startswith(("|", "#", " ")))
    except OSError:
        return None
    h = hashlib.sha256()
    for s in sources:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if fields.get("source_sha256") != h.hexdigest():
        return None
    return fields


def measured_traffic_bytes():
    """HBM bytes per construction launch from the committed counter summary,
    or None when the construction sources changed since it was taken."""
    f = counter_summary(TRAFFIC_FILE, TRAFFIC_SOURCES)
    return None if f is None else float(f["stage_traffic_bytes_per_launch"])


def batched_bytes_per_iteration(sizes, m: int, k: int) -> int:
    """Algorithmic bytes of one iteration of the batched colonies: per ant-step
    the row (8k), tour entry, slot and the edge's distance (9 B, as the single
    instance); per tour edge the deposit (tour entry, slot, reverse slot and
    one int64 atomic on the canonical slot, written back: 22 B); per candidate
    slot the merge, the cleared sum and the next choice weights (32 B)."""
    sizes = np.asarray(sizes, np.int64)
    steps = int((m * (sizes - 1)).sum())
    edges = int((m * sizes).sum())
    slots = int(sizes.sum()) * k
    return steps * (8 * k + 9) + edges * 22 + slots * 32


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(xy, cfg, tau0_gpu, threads, ants_per_thread=4):
    """Oracle construction of a fixed sample of ants (iteration 0) on the host."""
    import oracle as orc
    n, k = len(xy), cfg["k"]
    t0 = time.time()
    nn, nnd = orc.knn_rows(xy, k, threads=threads)
    t_knn = time.time() - t0
    t0 = time.time()
    L_nn = orc.nn_tour(xy, nn, nnd)[1]
    t_nn = time.time() - t0
    tau = np.full((n, k), orc.tau0(n, L_nn), np.float32)
    count = ants_per_thread * threads
    t0 = time.time()
    res = orc.construct(xy, nn, nnd, tau, cfg["alpha"], cfg["beta"], cfg["seed"], 0,
                        np.arange(count), threads=threads)
    dt = time.time() - t0
    # one thread, one ant: the oracle's single-core rate
    t1 = time.time()
    orc.construct(xy, nn, nnd, tau, cfg["alpha"], cfg["beta"], cfg["seed"], 0, np.arange(1),
                  threads=1)
    one = (n - 1) / (time.time() - t1)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=count * (n - 1) / dt, unit="ant-steps/s", cores=threads, kind="oracle",
                one_thread=one, cpu_model=model, cpu_count=os.cpu_count(),
                sample=f"{count} ants of iteration 0 at n={n} (FP64, O(n) fallback), "
                       f"{dt:.1f} s; candidate lists took {t_knn:.1f} s and are not counted",
                L_nn=L_nn, first_tour_s=t_knn + t_nn,
                tau0_matches_gpu=bool(orc.tau0(n, L_nn) == np.float32(tau0_gpu)),
                sample_best_len=int(res["lengths"].min()),
                fallback_share=float(res["fallbacks"].sum() / (count * (n - 1))))


def deposit_atomics(col) -> int:
    """Atomics one pheromone update issues for the colony's current tours: one
    per tour edge {i, j} with j in nn[i] or i in nn[j] (its canonical slot)."""
    import torch
    tours = col.tours.long()
    nxt = torch.roll(tours, -1, dims=1)
    fwd = torch.zeros_like(tours, dtype=torch.bool)
    fwd[:, :-1] = col.slots[:, 1:] != 255            # recorded candidate moves
    i, j = tours[~fwd], nxt[~fwd]                     # fallback moves and closing edges
    nn = col.nn.long()
    hit = torch.zeros(i.numel(), dtype=torch.bool, device=i.device)
    for c0 in range(0, i.numel(), 1 << 22):
        a, b = i[c0:c0 + (1 << 22)], j[c0:c0 + (1 << 22)]
        hit[c0:c0 + a.numel()] = ((nn[a] == b[:, None]).any(1) | (nn[b] == a[:, None]).any(1))
    return int(fwd.sum().item() + hit.sum().item())


def equal_time_block(name, threads):
    """Equal-time and equal-iteration comparison on a workload the oracle runs
    to completion (n = 1,000 and n = 20,000 uniform).

    Both sides run the same loop with the same Philox keys: NN-tour
    initialisation, then every iteration (construction, best tracking,
    update).  Candidate lists are built first on both sides and not counted
    (the oracle's are an O(n^2) brute force).  The best so far is stamped
    after each iteration on each side's own clock.  T is the GPU's time for
    the whole loop; the oracle's best at T is the best it had reached by
    then (its NN tour once built).  The equal-iteration figures compare the
    final bests, and the oracle's time to finish against the GPU's."""
    import torch

    import oracle as orc
    import paper_1709_03187_amd as aco
    from paper_1709_03187_amd import instances

    cfg = instances.CONFIGS[name]
    xy = instances.make_coords(name)
    n, m, k, iters = cfg["n"], cfg["m"], cfg["k"], cfg["iterations"]
    # GPU
    col = aco.Colony(xy=xy, k=k, m=m, alpha=cfg["alpha"], beta=cfg["beta"], rho=cfg["rho"],
                     seed=cfg["seed"])
    col.build_candidates()
    torch.cuda.synchronize()
    t0 = time.time()
    col.init_pheromone()
    torch.cuda.synchronize()
    gpu_marks = [(time.time() - t0, col.L_nn)]
    for it in range(iters):
        col.iterate(it)
        torch.cuda.synchronize()
        gpu_marks.append((time.time() - t0, int(col.best_len.item())))
    T = gpu_marks[-1][0]
    gpu_best = gpu_marks[-1][1]
    del col
    torch.cuda.empty_cache()
    # oracle
    t0 = time.time()
    nn, nnd = orc.knn_rows(xy, k, threads=threads)
    knn_s = time.time() - t0
    t0 = time.time()
    L_nn = orc.nn_tour(xy, nn, nnd)[1]
    tau = np.full((n, k), orc.tau0(n, L_nn), np.float32)
    best = L_nn
    or_marks = [(time.time() - t0, best)]
    for it in range(iters):
        r = orc.construct(xy, nn, nnd, tau, cfg["alpha"], cfg["beta"], cfg["seed"], it,
                          np.arange(m), threads=threads)
        tau = orc.update(nn, tau, r["tours"], r["lengths"], cfg["rho"], 32, threads=threads)
        best = min(best, int(r["lengths"].min()))
        or_marks.append((time.time() - t0, best))
        log(f"[bench] {name} oracle iteration {it} done ({or_marks[-1][0]:.1f} s)")
    at_T = [mk for mk in or_marks if mk[0] <= T]
    or_best_T = at_T[-1][1] if at_T else None
    or_best = or_marks[-1][1]
    return {
        "workload": f"n={n:,} uniform integer cities in [0,1e6]^2, m={m}, k={k}, alpha=1, "
                    f"beta=2, rho=0.1, {iters} iterations, Philox seed {cfg['seed']}",
        "equal_time": {
            "seconds": T, "gpu_best": gpu_best,
            "oracle_best": or_best_T,
            "oracle_iterations_done": max(0, len(at_T) - 1),
            "gap": None if or_best_T is None else (gpu_best - or_best_T) / or_best_T},
        "equal_iterations": {
            "iterations": iters, "gpu_best": gpu_best, "oracle_best": or_best,
            "gap": (gpu_best - or_best) / or_best,
            "gpu_seconds": T, "oracle_seconds": or_marks[-1][0],
            "oracle_over_gpu_time": or_marks[-1][0] / T},
        "gpu_best_by_iteration": [v for _, v in gpu_marks],
        "oracle_best_by_iteration": [v for _, v in or_marks],
        "candidate_lists_not_counted_s": {"oracle": knn_s},
        "oracle_threads": threads,
    }


def batched_block():
    """The batched workload: 4,096 instances, n log-uniform in [100, 5,000],
    m = 64, k = 12, 30 iterations, one persistent launch per run.  The first
    run tunes waves-per-instance and the visited layout; the timed run
    repeats the 30 iterations from a fresh set-up with the tuned values."""
    import torch

    import paper_1709_03187_amd as aco
    from paper_1709_03187_amd import instances

    cfg = instances.CONFIGS["c4"]
    xy, off, sizes = instances.make_batched("c4")
    iters = cfg["iterations"]
    bt = aco.Batch(xy, off, k=cfg["k"], m=cfg["m"], alpha=cfg["alpha"], beta=cfg["beta"],
                   rho=cfg["rho"], seed=cfg["seed"], iterations=iters)
    torch.cuda.synchronize()
    t0 = time.time()
    tuned = bt.run(autotune=1)
    torch.cuda.synchronize()
    t_tuned_run = time.time() - t0
    t0 = time.time()
    bt.setup()
    torch.cuda.synchronize()
    t_setup = time.time() - t0
    ib = torch.empty((bt.B, iters), dtype=torch.int64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    bt.iterate(0, iters, waves=tuned[0], layout=tuned[1], iter_best=ib, occupancy=tuned[2])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    steps = int(cfg["m"] * (sizes - 1).sum()) * iters
    L0 = bt.best_lens.cpu().numpy()
    alg = batched_bytes_per_iteration(sizes, cfg["m"], cfg["k"]) * iters
    achieved = alg / (ms * 1e-3) / 1e9
    cs = counter_summary(BATCH_TRAFFIC_FILE, BATCH_TRAFFIC_SOURCES)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if cs is None else float(cs["launch_traffic_bytes"]) / (ms * 1e-3) / 1e9,
            "l2_hit_rate": None if cs is None else float(cs["l2_hit_rate"]),
            "kernel": "k_b_colony (all 30 iterations: construction, lengths, deposit, merge, "
                      "choice weights)",
            "algorithmic_bytes_per_launch": alg,
            "traffic_bytes_per_launch": None if cs is None else float(cs["launch_traffic_bytes"])}
    return {"workload": f"{bt.B} instances, n log-uniform in [100, 5000] (sum {bt.N}), m=64, "
                        f"k=12, 30 iterations, one persistent launch",
            "ant_steps_per_s": steps / (ms * 1e-3), "launch_ms": ms, "roofline": roof,
            "ms_per_iteration": ms / iters, "setup_ms": t_setup * 1e3,
            "first_run_with_tuning_s": t_tuned_run,
            "tuned": {"waves_per_instance": tuned[0],
                      "visited_layout": {1: "bits", 2: "bytes", 3: "bits"}[tuned[1]],
                      "ants_per_wave": 4 if tuned[1] == 3 else 1,
                      "waves_per_simd": tuned[2]},
            "mean_best_len": float(L0.mean())}


MLP_FLOP_FORWARD = 2 * (8 * 64 + 64 * 64 + 64)          # per edge: three layers
MLP_FLOP_BACKWARD = MLP_FLOP_FORWARD + 2 * (64 + 64 * 64 + 64 * 64 + 64 * 8)  # + dW3, d1, dW2, dW1
MFMA_BF16_PEAK_TFLOPS = 2500.0


def _timed(fn, reps):
    """Mean milliseconds of fn() over reps launches, HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _colony_until(xy, cfg, beta, budget_s, iterations, theta=None):
    """Best length of a colony run within budget_s seconds (set-up included)."""
    import torch

    import paper_1709_03187_amd as aco
    col = aco.Colony(xy=xy, k=cfg["k"], m=cfg["m"], alpha=cfg["alpha"], beta=beta,
                     rho=cfg["rho"], seed=cfg["seed"], theta=theta)
    torch.cuda.synchronize()
    t0 = time.time()
    col.setup()
    torch.cuda.synchronize()
    setup = time.time() - t0
    it = 0
    while it < iterations:
        t_it = time.time()
        col.iterate(it)
        torch.cuda.synchronize()
        it += 1
        # stop where one more iteration (as long as the last) would pass the budget
        if budget_s is not None and time.time() + (time.time() - t_it) > t0 + budget_s:
            break
    res = dict(best_len=int(col.best_len.item()), iterations=it, seconds=time.time() - t0,
               setup_s=setup, L_nn=col.L_nn)
    del col
    torch.cuda.empty_cache()
    return res


LEARNED_BETAS = (2.0, 4.0, 8.0, 12.0)


def learned_block(xy_eval, cfg):
    """Learned heuristic: 64 uniform n=20,000 instances (seeds 1000..1063) are
    solved by the batched colonies (m=64, k=16, 30 iterations, beta=2) and
    each best tour is made 2-optimal within a window of 1,000 positions; its
    candidate edges are the positive labels.  3,000 Adam steps of 65,536
    edges train the network.  Each heuristic (plain eta = 1/d, learned score)
    then gets its own best beta from {2, 4, 8, 12}, chosen on two held-out
    uniform n=20,000 instances (m=256, 30 iterations); on the evaluation
    workload plain eta at its beta runs its 20 iterations (wall clock T, set-up
    included) and the learned score at its beta runs for the same T.  Plain
    eta at the learned score's beta, and both at beta=2, run for T beside
    them."""
    import torch

    import paper_1709_03187_amd as aco
    from paper_1709_03187_amd import instances, learned

    k = cfg["k"]
    xys = [instances.uniform_coords(20000, 1000 + b) for b in range(64)]
    data = learned.training_set(xys, k=k, m=64, iterations=30, seed=1, two_opt_window=1000)
    E = int(data.feat.shape[0])
    set_s = data.seconds
    train_steps, train_batch = 3000, 65536
    tr = learned.train(data, instances.mlp_parameters(0), steps=train_steps, batch=train_batch,
                       lr=2e-3, log_every=1000)
    theta = tr.theta
    # kernel rates: backward on one training batch, forward on the evaluation edges
    B = train_batch
    grad = torch.empty(aco.ACO_MLP_PARAMS, dtype=torch.float32, device="cuda")
    ws = torch.empty(aco.aco_mlp_backward_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    bwd_ms = _timed(lambda: aco.aco_mlp_backward(data.feat[:B], data.labels[:B], B, theta, 1.0,
                                                 grad, None, ws), 50)
    del data, ws
    col = aco.Colony(xy=xy_eval, k=k, m=8, beta=8.0)
    col.build_candidates()
    feat = col.features()
    Ev = col.n * k
    fwd_ms = _timed(lambda: aco.aco_mlp_forward(feat, Ev, theta, aco.ACO_MLP_OUT_ETA_B, 8.0,
                                                col.eta_b), 50)
    fws = torch.empty(aco.aco_features_workspace_bytes(), dtype=torch.uint8, device="cuda")
    feat_ms = _timed(lambda: aco.aco_edge_features(col.xy, col.n, k, col.nn, col.nnd, col.rev,
                                                   feat, fws), 20)
    del col, feat
    torch.cuda.empty_cache()
    # beta chosen per heuristic on held-out instances
    held = [instances.uniform_coords(20000, 5000 + b) for b in range(2)]
    hcfg = dict(cfg, m=256)
    sel = {"plain": {}, "learned": {}}
    for beta in LEARNED_BETAS:
        for name, th in (("plain", None), ("learned", theta)):
            sel[name][beta] = float(np.mean([_colony_until(x, hcfg, beta, None, 30, theta=th)
                                             ["best_len"] for x in held]))
    b_plain = min(LEARNED_BETAS, key=lambda b: sel["plain"][b])
    b_lrn = min(LEARNED_BETAS, key=lambda b: sel["learned"][b])
    its = cfg["iterations"]
    plain = _colony_until(xy_eval, cfg, b_plain, None, its)
    T = plain["seconds"]
    lrn = _colony_until(xy_eval, cfg, b_lrn, T, 100 * its, theta=theta)
    plain_same = _colony_until(xy_eval, cfg, b_lrn, T, 100 * its)
    plain2 = _colony_until(xy_eval, cfg, 2.0, T, 100 * its)
    lrn2 = _colony_until(xy_eval, cfg, 2.0, T, 100 * its, theta=theta)
    fwd_tflops = MLP_FLOP_FORWARD * Ev / (fwd_ms * 1e-3) / 1e12
    bwd_tflops = MLP_FLOP_BACKWARD * B / (bwd_ms * 1e-3) / 1e12

    def gain(ref, x):
        return (ref["best_len"] - x["best_len"]) / ref["best_len"]
    return {
        "training": {"instances": 64, "n": 20000, "edges": E,
                     "label_colony": "batched, m=64, k=16, beta=2, 30 iterations, best tours "
                                     "2-optimal within 1,000 positions",
                     "set_build_s": set_s, "steps": train_steps, "batch": train_batch,
                     "lr": 2e-3,
                     "train_s": tr.seconds, "train_steps_s": tr.steps_seconds,
                     "loss": tr.losses,
                     # end to end over the training steps: backward flops of
                     # every step's batch over the steps' wall clock (the
                     # reductions, Adam and launches included)
                     "roofline": {"bound": "mfma",
                                  "achieved": MLP_FLOP_BACKWARD * train_batch * train_steps
                                  / tr.steps_seconds / 1e12,
                                  "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": MLP_FLOP_BACKWARD * train_batch * train_steps
                                  / tr.steps_seconds / 1e12 / MFMA_BF16_PEAK_TFLOPS}},
        "kernels": {
            "mlp_forward": {"edges": Ev, "ms": fwd_ms, "flop_per_edge": MLP_FLOP_FORWARD,
                            "tflops": fwd_tflops, "peak_bf16_tflops": MFMA_BF16_PEAK_TFLOPS,
                            "frac": fwd_tflops / MFMA_BF16_PEAK_TFLOPS},
            "mlp_backward": {"edges": B, "ms": bwd_ms, "flop_per_edge": MLP_FLOP_BACKWARD,
                             "tflops": bwd_tflops, "frac": bwd_tflops / MFMA_BF16_PEAK_TFLOPS},
            "edge_features": {"edges": Ev, "ms": feat_ms}},
        "beta_selection_held_out": {"instances": "2 x n=20,000 uniform (seeds 5000, 5001), "
                                                 "m=256, k=16, 30 iterations, mean best",
                                    "plain": {f"{b:g}": v for b, v in sel["plain"].items()},
                                    "learned": {f"{b:g}": v for b, v in sel["learned"].items()},
                                    "best_beta_plain": b_plain, "best_beta_learned": b_lrn},
        "equal_wall_clock": {
            "seconds": T, "plain_best_beta": plain, "learned_best_beta": lrn,
            "plain_at_learned_beta": plain_same, "plain_beta2": plain2, "learned_beta2": lrn2,
            "gain_each_at_best_beta": gain(plain, lrn),
            "gain_same_beta": gain(plain_same, lrn),
            "gain_beta2": gain(plain2, lrn2)},
    }


def partial_block(xy, cfg, budget_s, pheromone_kind="table", sampler=0, two_opt_p=0.0,
                  window=500):
    """PartialACO (Section 3.1, Algorithm 1) on the evaluation workload with
    the paper's 1% cap at 200K cities and p = 1: iteration 0 builds full
    tours (the local bests); every later iteration each ant rebuilds at most
    n/100 cities of its local best.  Reports the time of a partial iteration
    (construction + local bests + pheromone update), the rebuilt ant-steps per
    second, and the best tour reached within `budget_s` seconds (the plain
    colony's run time) from set-up.  pheromone_kind="table": the n x k table with
    evaporation and the iteration's deposits; "local_best": recomputed each
    iteration from the ants' local bests (the paper's P-ACO variant, base
    1/(n-1), delta 1/m).  sampler 1: Independent Roulette (Section 3).
    two_opt_p > 0: after each construction the tours drawn with that
    probability get windowed 2-opt (Sections 4-5: p = 0.001, W = 500)."""
    import torch

    import paper_1709_03187_amd as aco
    n = cfg["n"]
    M = max(1, n // 100)
    col = aco.Colony(xy=xy, k=cfg["k"], m=cfg["m"], alpha=cfg["alpha"], beta=cfg["beta"],
                     rho=cfg["rho"], seed=cfg["seed"])
    torch.cuda.synchronize()
    t0 = time.time()
    col.setup()
    base, delta = 1.0 / (n - 1), 1.0 / cfg["m"]

    def pheromone():
        if pheromone_kind == "table":
            col.update()
        else:
            col.pheromone_from_local_best(base, delta)

    opt = dict(calls=0, tours=0, moves=0, gain=0, seconds=0.0)

    def two_opt(it):
        if two_opt_p <= 0:
            return
        t = time.time()
        st = col.two_opt(it, p=two_opt_p, window=window)
        opt["seconds"] += time.time() - t
        opt["calls"] += 1
        opt["tours"] += st["selected"]
        opt["moves"] += st["moves"]
        opt["gain"] += st["gain"]

    col.construct_ex(0, sampler=sampler)
    two_opt(0)
    col.update_local_best()
    col.track_best()
    pheromone()
    torch.cuda.synchronize()
    first_s = time.time() - t0
    lb_first = float(col.lbest_len.double().mean().item())
    stream = torch.cuda.current_stream()
    its = 1
    ev = []
    while True:
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        t_it = time.time()
        e[0].record(stream)
        col.construct_ex(its, sampler=sampler, p_partial=1.0, max_modify=M, partial=True)
        e[1].record(stream)
        two_opt(its)
        col.update_local_best()
        col.track_best()
        e[2].record(stream)
        pheromone()
        e[3].record(stream)
        torch.cuda.synchronize()
        ev.append(e)
        its += 1
        if time.time() + (time.time() - t_it) > t0 + budget_s:
            break
    con = np.array([x[0].elapsed_time(x[1]) for x in ev])
    it_ms = np.array([x[0].elapsed_time(x[3]) for x in ev])
    # rebuilt steps per ant: E[r] = (M + 1) / 2
    steps = cfg["m"] * (M + 1) / 2
    res = {"pheromone": pheromone_kind, "sampler": ["roulette", "independent"][sampler], "cap": M, "p_partial": 1.0, "iterations": its, "seconds": time.time() - t0,
           "first_full_iteration_s": first_s,
           "ms_per_partial_iteration": float(it_ms.mean()),
           "construct_partial_ms": float(con.mean()),
           "rebuilt_ant_steps_per_s": steps / (con.mean() * 1e-3),
           "best_len": int(col.best_len.item()), "L_nn": col.L_nn,
           "mean_local_best_first": lb_first,
           "mean_local_best_last": float(col.lbest_len.double().mean().item())}
    if two_opt_p > 0:
        res["two_opt"] = dict(p=two_opt_p, window=window, **opt)
    del col
    torch.cuda.empty_cache()
    return res


def two_opt_block(xy, cfg, tours=4, window=500):
    """Windowed 2-opt (Sections 4-5) of `tours` constructed tours of the main
    workload at once (every tour takes part): wall time of the call, rounds,
    moves and the length reduction.  The first round evaluates every move:
    n (W - 1) per tour."""
    import torch

    import paper_1709_03187_amd as aco
    n = cfg["n"]
    col = aco.Colony(xy=xy, k=cfg["k"], m=tours, alpha=cfg["alpha"], beta=cfg["beta"],
                     rho=cfg["rho"], seed=cfg["seed"])
    col.setup()
    out = []
    for it in range(2):
        col.construct(it)
        L0 = col.lengths.double().sum().item()
        torch.cuda.synchronize()
        t = time.time()
        st = col.two_opt(it, p=1.0, window=window, batch=tours)
        torch.cuda.synchronize()
        out.append(dict(seconds=time.time() - t, **st,
                        length_reduction=-st["gain"] / L0))
    w = min(window, n // 2)
    res = {"tours": tours, "window": window, "runs": out,
           "first_round_move_evaluations": tours * n * (w - 1),
           "mean_len_after": float(col.lengths.double().mean().item()),
           "L_nn": col.L_nn}
    del col
    torch.cuda.empty_cache()
    return res


def independent_block(xy, cfg, iterations=3):
    """Full construction with Independent Roulette (Section 3) on the main
    workload: construction time per iteration and ant-steps/s, next to the
    roulette's."""
    import torch

    import paper_1709_03187_amd as aco
    col = aco.Colony(xy=xy, k=cfg["k"], m=cfg["m"], alpha=cfg["alpha"], beta=cfg["beta"],
                     rho=cfg["rho"], seed=cfg["seed"])
    col.setup()
    stream = torch.cuda.current_stream()
    ms = []
    for it in range(iterations + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        col.construct_ex(it, sampler=aco.ACO_SAMPLER_INDEPENDENT)
        e1.record(stream)
        col.track_best()
        col.update()
        torch.cuda.synchronize()
        if it > 0:
            ms.append(e0.elapsed_time(e1))
    steps = cfg["m"] * (cfg["n"] - 1)
    res = {"construct_ms": float(np.mean(ms)), "ant_steps_per_s": steps / (np.mean(ms) * 1e-3),
           "iterations_timed": iterations, "best_len": int(col.best_len.item())}
    del col
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=19)    # with the warm-up: the 20 iterations of the workload
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-partial", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the colony has no multi-GPU path "
              "(it would shard ants by index and all-reduce the int64 deposits).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1709_03187_amd as aco
    from paper_1709_03187_amd import instances

    cfg = instances.CONFIGS[WORKLOAD]
    n, m, k = cfg["n"], cfg["m"], cfg["k"]
    xy = instances.make_coords(WORKLOAD)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] {WORKLOAD}: n={n} m={m} k={k}")

    # calibration copy for the HBM traffic counters (known size, 256 MiB each way)
    src = torch.empty(64 * 2**20, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    col = aco.Colony(xy=xy, k=k, m=m, alpha=cfg["alpha"], beta=cfg["beta"], rho=cfg["rho"],
                     seed=cfg["seed"], device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.time()
    col.build_candidates()
    torch.cuda.synchronize()
    t_cand = time.time() - t0
    t0 = time.time()
    col.init_pheromone()
    torch.cuda.synchronize()
    t_init = time.time() - t0
    log(f"[bench] candidates {t_cand*1e3:.1f} ms, NN-tour init {t_init*1e3:.1f} ms, "
        f"L_nn={col.L_nn}")

    iters = args.warmup + args.steps
    iter_best = torch.empty(iters, dtype=torch.int64, device=dev)
    wall0 = time.time()
    for it in range(args.warmup):
        col.iterate(it, iter_best[it:it + 1])
        torch.cuda.synchronize()
        log(f"[bench] warmup iteration {it} done")
    wall_warm = time.time() - wall0

    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.time()
    for s in range(args.steps):
        it = args.warmup + s
        e = ev[s]
        e[0].record(stream)
        col.construct(it)
        e[1].record(stream)
        col.track_best(iter_best[it:it + 1])
        e[2].record(stream)
        col.update()
        e[3].record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    t_con = np.array([ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)])
    t_best = np.array([ev[s][1].elapsed_time(ev[s][2]) for s in range(args.steps)])
    t_upd = np.array([ev[s][2].elapsed_time(ev[s][3]) for s in range(args.steps)])
    t_step = np.array([ev[s][0].elapsed_time(ev[s][3]) for s in range(args.steps)])
    for s in range(args.steps):
        log(f"[bench] step {s}: construct {t_con[s]:.2f} ms, best {t_best[s]:.3f} ms, "
            f"update {t_upd[s]:.2f} ms")

    steps_per_iter = m * (n - 1)
    ms_per_step = float(t_step.mean())
    value = steps_per_iter / (ms_per_step * 1e-3)
    bps = construct_bytes_per_step(k)
    launch_s = t_con.mean() * 1e-3
    achieved = construct_bytes_per_launch(n, m, k) / launch_s / 1e9
    tb = measured_traffic_bytes()
    traffic = None if tb is None else tb / launch_s / 1e9
    ib = iter_best.cpu().numpy()
    best_len = int(col.best_len.item())
    atomics = deposit_atomics(col)

    out = {
        "metric": "ant construction steps/sec at n=200K",
        "value": value,
        "unit": "ant-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        # the roulette's running sums and draw are FP64; the rest of the path is
        # not: weights and pheromone are FP32, the deposit is int64 fixed point
        "dtype_detail": {"roulette_sums": "f64", "choice_weights": "f32", "pheromone": "f32",
                         "deposit": "int64 fixed point (2^-32)", "lengths": "int64"},
        "data": "synthetic",
        "config": {"workload": "n=200,000 clustered cities (100 Gaussian clusters, sigma=1e4, "
                               "integer coords), m=1,024 ants, k=16, alpha=1, beta=2, rho=0.1, "
                               "int64 fixed-point deposit (2^-32), Philox seed 3",
                   "n": n, "m": m, "k": k, "iterations_timed": args.steps,
                   "parallelism": "one ant per wavefront"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "aco_construct_tours (k_choice_info + k_construct)",
                     "bytes_per_ant_step": bps,
                     "algorithmic_bytes_per_launch": construct_bytes_per_launch(n, m, k),
                     "traffic_bytes_per_launch": tb},
        "construct_ms": float(t_con.mean()),
        "update_ms": float(t_upd.mean()),
        "deposit": {"atomics_per_launch": atomics,
                    "atomics_per_s": atomics / (t_upd.mean() * 1e-3),
                    "atomic_rate_probe_per_s": ATOMIC_RATE_PROBE,
                    "frac_of_probe": atomics / (t_upd.mean() * 1e-3) / ATOMIC_RATE_PROBE,
                    "note": "one int64 atomic per tour edge with a candidate slot (the last "
                            "iteration's tours); update_ms also holds the merge and quanta"},
        "best_ms": float(t_best.mean()),
        "construct_ant_steps_per_s": steps_per_iter / (t_con.mean() * 1e-3),
        "setup_ms": {"candidates": t_cand * 1e3, "nn_tour_init": t_init * 1e3},
        "wall_s_timed": wall,
        "L_nn": col.L_nn,
        "iter_best": [int(v) for v in ib],
        "best_len": best_len,
    }
    tau0_gpu = col.tau0
    del col
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("[bench] batched workload")
        out["batched"] = batched_block()
    if not args.no_learned:
        log("[bench] learned heuristic: training and equal-time comparison")
        out["learned"] = learned_block(xy, cfg)
    if not args.no_partial:
        log("[bench] PartialACO at the 1% cap")
        gpu_time = t_cand + t_init + wall_warm + wall
        out["partial"] = partial_block(xy, cfg, gpu_time)
        out["partial"]["plain_best_len_same_time"] = best_len
        log("[bench] PartialACO on local-best pheromone")
        out["partial_local_best_pheromone"] = partial_block(xy, cfg, gpu_time, "local_best")
        log("[bench] the paper's method: PartialACO + Independent Roulette + local-best pheromone")
        out["partial_independent_local_best"] = partial_block(xy, cfg, gpu_time, "local_best", 1)
        log("[bench] Independent Roulette, full tours")
        out["independent_roulette"] = independent_block(xy, cfg)
        log("[bench] windowed 2-opt of constructed tours")
        out["two_opt"] = two_opt_block(xy, cfg)
        log("[bench] PartialACO + Independent Roulette + local-best pheromone + 2-opt")
        out["partial_independent_local_best_two_opt"] = partial_block(
            xy, cfg, gpu_time, "local_best", 1, two_opt_p=0.001, window=500)
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or max(1, min(16, os.cpu_count() or 1))
        for name in ("c1", "c2"):
            log(f"[bench] {name}: GPU and oracle runs to completion, {threads} threads")
            out[f"equal_time_{name}"] = equal_time_block(name, threads)
        log(f"[bench] cpu baseline with {threads} threads")
        cb = cpu_baseline(xy, cfg, tau0_gpu, threads)
        out["cpu_baseline"] = {kk: cb[kk] for kk in ("value", "unit", "cores", "kind", "sample")}
        # equal wall time T = the GPU's whole run (set-up, warm-up and timed iterations).
        # Within T the oracle has at best its nearest-neighbour tour (one iteration of
        # construction takes it m(n-1)/rate seconds); before its set-up ends it has none.
        gpu_time = t_cand + t_init + wall_warm + wall
        oracle_has_tour = cb["first_tour_s"] <= gpu_time
        oracle_iter_s = m * (n - 1) / cb["value"]
        out["equal_time"] = {
            "seconds": gpu_time, "gpu_best": best_len,
            "oracle_first_tour_s": cb["first_tour_s"],
            "oracle_seconds_per_iteration": oracle_iter_s,
            "oracle_best": cb["L_nn"] if oracle_has_tour else None,
            "gap": ((best_len - cb["L_nn"]) / cb["L_nn"]) if oracle_has_tour else None,
            "gap_vs_oracle_nn_tour_whenever_ready": (best_len - cb["L_nn"]) / cb["L_nn"],
        }
        comb = out.get("partial_independent_local_best_two_opt")
        if comb is not None:
            # the paper's combination (PartialACO, Independent Roulette, pheromone
            # from the local bests, 2-opt) ran for the same time from set-up
            out["equal_time"]["gpu_best_partial_ir_local_best_two_opt"] = comb["best_len"]
            out["equal_time"]["gap_partial_ir_local_best_two_opt_vs_oracle_nn_tour"] = (
                (comb["best_len"] - cb["L_nn"]) / cb["L_nn"])
        out["cpu_baseline_extra"] = {"tau0_matches_gpu": cb["tau0_matches_gpu"],
                                     "fallback_share": cb["fallback_share"],
                                     "sample_best_len": cb["sample_best_len"],
                                     "one_thread_ant_steps_per_s": cb["one_thread"],
                                     "cpu_model": cb["cpu_model"], "cpu_count": cb["cpu_count"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
