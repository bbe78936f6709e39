"""Learned edge heuristic: training data from the colony's own best tours,
training with the library's network kernels, and use in a colony.

Training pipeline (all arithmetic in libaco.so kernels; torch only holds
device memory and reorders rows):
  1. the batched colonies run on the training instances; their best tours
     label the candidate edges (1 = edge of the best tour);
  2. aco_edge_features gives the 8 features of every candidate edge;
  3. minibatches of a fixed random order of all edges go through
     aco_mlp_backward (fused forward + backward) and aco_mlp_adam, run on
     the device by aco_mlp_train between the logged steps.
The trained parameters are passed as `theta` to Colony, whose eta_b is then
sigmoid(score)^beta instead of (1/d)^beta.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import (ACO_MLP_PARAMS, Batch, aco_edge_features, aco_features_workspace_bytes,
               aco_mlp_backward, aco_mlp_backward_workspace_bytes, aco_mlp_train,
               aco_tour_edge_labels, aco_two_opt, aco_two_opt_workspace_bytes)


@dataclass
class TrainingSet:
    feat: object            # float32 [E, 8] (GPU)
    labels: object          # uint8 [E] (GPU)
    best_lens: np.ndarray   # best tour length per training instance
    seconds: float          # wall clock of colonies + features + labels


def training_set(xys, k=16, m=64, iterations=30, seed=1, stream=None, beta=2.0,
                 two_opt_window=0) -> TrainingSet:
    """Run the batched colonies on the instances `xys` (list of int32 [n, 2])
    and label every candidate edge by the best tour found; with
    two_opt_window > 0 each best tour is first made 2-optimal within that
    window (windowed 2-opt to convergence), so the labels come from better
    tours than the colony's own."""
    import torch
    t0 = time.perf_counter()
    sizes = np.array([len(x) for x in xys], np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bt = Batch(np.concatenate(xys), off, k=k, m=m, beta=beta, seed=seed, iterations=iterations)
    bt.run(autotune=0, stream=stream)
    N = bt.N
    if two_opt_window:
        tws = torch.empty(aco_two_opt_workspace_bytes(int(sizes.max()), 1, 1), dtype=torch.uint8,
                          device="cuda")
        for b in range(bt.B):
            lo, hi = int(off[b]), int(off[b + 1])
            aco_two_opt(bt.xy[lo:hi], hi - lo, 1, bt.best_tours[lo:hi], bt.best_lens[b:b + 1],
                        None, two_opt_window, 1.0, seed, 0, 0, 1, tws, stream)
    nn = bt.view("nn", torch.int32, N * k)
    nnd = bt.view("nnd", torch.int32, N * k)
    rev = bt.view("rev", torch.int8, N * k)
    feat = torch.empty((N * k, 8), dtype=torch.float32, device="cuda")
    labels = torch.empty(N * k, dtype=torch.uint8, device="cuda")
    fws = torch.empty(aco_features_workspace_bytes(), dtype=torch.uint8, device="cuda")
    pos = torch.empty(int(sizes.max()), dtype=torch.int32, device="cuda")
    xy = bt.xy
    for b in range(bt.B):
        lo, hi = int(off[b]), int(off[b + 1])
        n = hi - lo
        aco_edge_features(xy[lo:hi], n, k, nn[lo * k:hi * k], nnd[lo * k:hi * k],
                          rev[lo * k:hi * k], feat[lo * k:hi * k], fws, stream)
        aco_tour_edge_labels(n, k, nn[lo * k:hi * k], bt.best_tours[lo:hi],
                             labels[lo * k:hi * k], pos, stream)
    torch.cuda.synchronize()
    return TrainingSet(feat, labels, bt.best_lens.cpu().numpy(), time.perf_counter() - t0)


@dataclass
class TrainResult:
    theta: object                 # float32 [ACO_MLP_PARAMS] (GPU)
    losses: list = field(default_factory=list)   # (step, loss) samples
    seconds: float = 0.0          # the whole call
    steps_seconds: float = 0.0    # the training steps alone (after the set is reordered)


def train(data: TrainingSet, theta0, steps=2000, batch=65536, lr=2e-3, pos_weight=1.0,
          seed=0, log_every=100, stream=None) -> TrainResult:
    """Adam on minibatches of a fixed random order of all edges."""
    import torch
    t0 = time.perf_counter()
    E = data.feat.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    order = torch.randperm(E, generator=g).cuda()
    feat = data.feat[order].contiguous()
    labels = data.labels[order].contiguous()
    theta = torch.as_tensor(np.asarray(theta0, np.float32)).cuda().contiguous()
    m = torch.zeros(ACO_MLP_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    grad = torch.empty_like(m)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B = min(batch, E)
    ws = torch.empty(aco_mlp_backward_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    res = TrainResult(theta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the steps run on the device in runs that end at the logged steps (step s
    # takes the batch of edges ((s mod floor(E / B)) B, ...) of the fixed order)
    ends = sorted(set(range(0, steps, log_every)) | {steps - 1}) if log_every else [steps - 1]
    a = 0
    for b in ends:
        if b < a:
            continue
        aco_mlp_train(feat, labels, E, theta, m, v, pos_weight, a + 1, b - a + 1, B, lr, grad,
                      loss, ws, stream=stream)
        if log_every:
            res.losses.append((b, float(loss.item())))
        a = b + 1
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res.seconds = t2 - t0
    res.steps_seconds = t2 - t1
    return res


def mean_loss(data: TrainingSet, theta, pos_weight=1.0, batch=1 << 20) -> float:
    """Weighted mean BCE over the whole set (a backward pass per chunk)."""
    import torch
    E = data.feat.shape[0]
    grad = torch.empty(ACO_MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(aco_mlp_backward_workspace_bytes(min(batch, E)), dtype=torch.uint8,
                     device="cuda")
    total = 0.0
    for lo in range(0, E, batch):
        n = min(batch, E - lo)
        aco_mlp_backward(data.feat[lo:lo + n], data.labels[lo:lo + n], n, theta, pos_weight,
                         grad, loss, ws)
        total += float(loss.item()) * n
    return total / E
