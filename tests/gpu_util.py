"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
check it against the CPU oracle (teacher-forced replay, bit-exact update)."""
from __future__ import annotations

import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as orc

BOUNDARY_EPS = 1e-6      # |u - C_r/S| window inside which the two sides may choose differently
BOUNDARY_RATE = 1e-4     # allowed share of such steps
PROB_RTOL = 1e-5         # choice probabilities, relative


def threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def colony(xy, k, m, **kw):
    import paper_1709_03187_amd as aco
    return aco.Colony(xy=xy, k=k, m=m, **kw)


def to_np(t):
    return t.detach().cpu().numpy()


def replay_ants(xy, nn, nnd, tau, alpha, beta, seed, iteration, tours, ants, eta=None,
                sweep=None):
    """Replay every given GPU tour with the oracle; returns (per-ant counts, probs)."""
    def one(q):
        return orc.replay(xy, nn, nnd, tau, alpha, beta, seed, iteration, int(ants[q]), tours[q],
                          eta=eta, boundary_eps=BOUNDARY_EPS, sweep=sweep)
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        res = list(ex.map(one, range(len(ants))))
    return [r[0] for r in res], np.stack([r[1] for r in res])


def check_tours(xy, nn, nnd, tau, alpha, beta, seed, iteration, tours, lengths, slots, probs,
                ants, eta=None, label="", sweep=None):
    """Full parity check of GPU tours for one iteration.  Returns the summed counts.
    sweep: the oracle's x_sweep_index, to check fallback moves by its sweep along x
    (same city as its brute force) instead of the O(n) scan."""
    n = len(xy)
    k = nn.shape[1]
    counts, oprob = replay_ants(xy, nn, nnd, tau, alpha, beta, seed, iteration, tours, ants, eta,
                                sweep)
    tot = {f: sum(c[f] for c in counts) for f in counts[0]}
    assert tot["invalid"] == 0, (label, tot)
    assert tot["hard_mismatch"] == 0, (label, tot)
    assert tot["fallback_mismatch"] == 0, (label, tot)
    assert tot["near_boundary_mismatch"] <= BOUNDARY_RATE * max(tot["steps"], 1) + 0, (label, tot)
    for q in range(len(ants)):
        T = tours[q]
        assert np.array_equal(np.sort(T), np.arange(n)), f"{label}: ant {ants[q]} not a permutation"
        assert lengths[q] == orc.tour_length(xy, T), f"{label}: ant {ants[q]} length"
        sl = slots[q]
        assert sl[0] == 255
        fb = sl[1:] == 255
        # fallback steps coincide with the oracle's fallback steps
        assert np.array_equal(fb, oprob[q, 1:] < 0), f"{label}: ant {ants[q]} fallback pattern"
        idx = np.nonzero(~fb)[0] + 1
        assert np.all(sl[idx] < k)
        assert np.array_equal(nn[T[idx - 1], sl[idx]], T[idx]), f"{label}: slot record"
        if probs is not None:
            p_gpu = probs[q, idx].astype(np.float64)
            p_or = oprob[q, idx]
            ok = np.abs(p_gpu - p_or) <= PROB_RTOL * p_or
            assert ok.all(), (label, ants[q], np.max(np.abs(p_gpu - p_or) / p_or))
            assert np.all(probs[q, np.nonzero(fb)[0] + 1] == -1.0)
    return tot
