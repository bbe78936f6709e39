"""CPU oracle for the ACO hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does: it shares no code,
header, table or helper with anything here.

Thin ctypes wrapper around `aco_oracle.c` (plain C, FP64, brute-force
fallback).  Every function mirrors a step of the method:

* distances: nint of the Euclidean distance (Section 2, the symmetric TSP);
* candidate lists: k smallest (d, j) per city (Section 6, ACS candidate lists);
* Philox4x32-10 draws keyed by (seed, iteration, ant, step);
* construction with the random proportional rule (Section 2, Eq. 1);
* evaporation then all-ant deposit (Section 2, Eq. 2-4) in int64 fixed point.

Parity status of each function is listed in `PINS` below.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aco_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# Which test pins each oracle function (all pinned; see tests/test_oracle_*.py).
PINS = {
    "nint_sqrt": "exhaustive s <= 2e6 and random s < 2^62 against math.isqrt",
    "knn_rows": "numpy lexsort brute force; scipy cKDTree",
    "rev": "numpy search of the transposed lists",
    "philox4x32_10": "rocRAND's philox4x32_10 ten_rounds (library routine, compiled from its header)",
    "nearest_unvisited": "plain argmin of (nint d, j) and numpy brute force",
    "nearest_unvisited_sweep": "the brute-force argmin on random visited sets (ties, duplicates, "
                               "equal x, negative coordinates, the clustered 200K instance)",
    "nn_tour": "plain O(n^2) argmin walk",
    "construct/replay": "exact rational probabilities (fractions); exhaustive tour enumeration (n<=7); "
                        "uniform permutations for alpha=beta=0, k=n-1; invariants",
    "update": "pure-evaporation closed form; numpy float32 merge; integer conservation; symmetry",
    "partial (PartialACO)": "p=0 equals the full construction; r=1 gives the rotated local best; "
                            "exact rational completion probabilities (n=7); plan statistics",
    "pheromone_local_best": "closed form for one tour; exact rational weights; conservation; "
                            "order invariance; the global best's weight is 2^shift",
}


def build(force: bool = False) -> str:
    """Compile aco_oracle.c into liboracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        i64, i32, u64, dbl, p = C.c_int64, C.c_int32, C.c_uint64, C.c_double, C.c_void_p
        sigs = {
            "oracle_sq": (i64, [p, i64, i64]),
            "oracle_nint_sqrt": (i64, [i64]),
            "oracle_dist": (i64, [p, i64, i64]),
            "oracle_tour_length": (i64, [p, i64, p]),
            "oracle_knn_rows": (None, [p, i64, C.c_int, p, i64, p, p]),
            "oracle_knn_rows_mt": (None, [p, i64, C.c_int, p, i64, p, p, C.c_int]),
            "oracle_rev": (None, [i64, C.c_int, p, p]),
            "oracle_philox4x32_10": (None, [p, p, p]),
            "oracle_draw": (C.c_uint32, [u64, i64, i64, i64]),
            "oracle_start_city": (i64, [u64, i64, i64, i64]),
            "oracle_nearest_unvisited": (i64, [p, i64, i64, p]),
            "oracle_nearest_unvisited_plain": (i64, [p, i64, i64, p]),
            "oracle_nn_tour": (i64, [p, i64, C.c_int, p, p, p]),
            "oracle_nn_tour_plain": (i64, [p, i64, p]),
            "oracle_tau0": (C.c_float, [i64, i64]),
            "oracle_construct": (None, [i64, C.c_int, p, p, p, p, p, dbl, dbl, u64, i64, p, i64,
                                        p, p, p, p, p, C.c_int]),
            "oracle_nearest_unvisited_sweep": (i64, [p, i64, i64, p, p, p]),
            "oracle_replay": (None, [i64, C.c_int, p, p, p, p, p, dbl, dbl, u64, i64, i64, p, dbl,
                                     p, p, p, p]),
            "oracle_deposit": (None, [i64, C.c_int, p, i64, p, p, C.c_int, p, C.c_int]),
            "oracle_update": (None, [i64, C.c_int, p, p, i64, p, p, dbl, C.c_int, C.c_int]),
            "oracle_run": (C.c_int, [i64, C.c_int, p, i64, dbl, dbl, dbl, i64, u64, C.c_int,
                                     C.c_int, p, p, p, p]),
            "oracle_partial_plan": (None, [u64, i64, i64, i64, u64, i64, p, p, p]),
            "oracle_pheromone_local_best": (None, [i64, C.c_int, p, i64, p, p, dbl, dbl,
                                                   C.c_int, p, p]),
            "oracle_construct_partial": (None, [i64, C.c_int, p, p, p, p, p, dbl, dbl, u64, i64,
                                                p, i64, p, u64, i64, C.c_int, p, p, p, p]),
            "oracle_replay_partial": (None, [i64, C.c_int, p, p, p, p, p, dbl, dbl, u64, i64, i64,
                                             p, u64, i64, C.c_int, p, dbl, p, p]),
            "oracle_two_opt_selected": (C.c_int, [u64, i64, i64, u64]),
            "oracle_two_opt_best": (None, [p, i64, p, i64, p, p]),
            "oracle_two_opt": (i64, [p, i64, p, i64, i64, p, p, p]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _xy(xy) -> np.ndarray:
    a = np.ascontiguousarray(xy, dtype=np.int32)
    assert a.ndim == 2 and a.shape[1] == 2
    return a


def _threads(threads: int | None) -> int:
    return int(threads) if threads else (os.cpu_count() or 1)


# ---------------------------------------------------------------- distances
def nint_sqrt(s: int) -> int:
    return int(lib().oracle_nint_sqrt(int(s)))


def dist(xy, i: int, j: int) -> int:
    xy = _xy(xy)
    return int(lib().oracle_dist(_p(xy), int(i), int(j)))


def tour_length(xy, tour) -> int:
    xy = _xy(xy)
    t = np.ascontiguousarray(tour, dtype=np.int32)
    return int(lib().oracle_tour_length(_p(xy), len(xy), _p(t)))


# ---------------------------------------------------------------- candidates
def knn_rows(xy, k: int, rows=None, threads=1):
    """(nn, nnd) int32 [len(rows)][k] for the requested cities (default: all)."""
    xy = _xy(xy)
    n = len(xy)
    assert 1 <= k <= min(n - 1, 64)
    rows = np.arange(n, dtype=np.int32) if rows is None else np.ascontiguousarray(rows, np.int32)
    nn = np.empty((len(rows), k), np.int32)
    nnd = np.empty((len(rows), k), np.int32)
    if threads == 1:
        lib().oracle_knn_rows(_p(xy), n, k, _p(rows), len(rows), _p(nn), _p(nnd))
    else:
        lib().oracle_knn_rows_mt(_p(xy), n, k, _p(rows), len(rows), _p(nn), _p(nnd),
                                 _threads(threads))
    return nn, nnd


def rev(nn) -> np.ndarray:
    nn = np.ascontiguousarray(nn, np.int32)
    n, k = nn.shape
    out = np.empty((n, k), np.int8)
    lib().oracle_rev(n, k, _p(nn), _p(out))
    return out


# ---------------------------------------------------------------- random numbers
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, iteration: int, ant: int, step: int) -> int:
    return int(lib().oracle_draw(seed, iteration, ant, step))


def start_city(seed: int, iteration: int, ant: int, n: int) -> int:
    return int(lib().oracle_start_city(seed, iteration, ant, n))


# ---------------------------------------------------------------- fallback / init
def nearest_unvisited(xy, c: int, visited, plain: bool = False) -> int:
    xy = _xy(xy)
    v = np.ascontiguousarray(visited, np.uint8)
    f = lib().oracle_nearest_unvisited_plain if plain else lib().oracle_nearest_unvisited
    return int(f(_p(xy), len(xy), int(c), _p(v)))


def x_sweep_index(xy):
    """(xorder, xpos): the cities by ascending x and each city's place in that order,
    for the sweep form of the nearest-unvisited search used when checking long tours."""
    xy = _xy(xy)
    order = np.argsort(xy[:, 0], kind="stable").astype(np.int32)
    pos = np.empty(len(xy), np.int32)
    pos[order] = np.arange(len(xy), dtype=np.int32)
    return order, pos


def nearest_unvisited_sweep(xy, c: int, visited, index=None) -> int:
    """The nearest unvisited city by a sweep along x (same result as the brute force)."""
    xy = _xy(xy)
    order, pos = x_sweep_index(xy) if index is None else index
    v = np.ascontiguousarray(visited, np.uint8)
    return int(lib().oracle_nearest_unvisited_sweep(_p(xy), len(xy), int(c), _p(v), _p(order),
                                                     _p(pos)))


def nn_tour(xy, nn, nnd):
    xy = _xy(xy)
    nn = np.ascontiguousarray(nn, np.int32)
    nnd = np.ascontiguousarray(nnd, np.int32)
    tour = np.empty(len(xy), np.int32)
    L = lib().oracle_nn_tour(_p(xy), len(xy), nn.shape[1], _p(nn), _p(nnd), _p(tour))
    return tour, int(L)


def nn_tour_plain(xy):
    xy = _xy(xy)
    tour = np.empty(len(xy), np.int32)
    L = lib().oracle_nn_tour_plain(_p(xy), len(xy), _p(tour))
    return tour, int(L)


def tau0(n: int, L_nn: int) -> np.float32:
    return np.float32(lib().oracle_tau0(int(n), int(L_nn)))


# ---------------------------------------------------------------- construction
def construct(xy, nn, nnd, tau, alpha, beta, seed, iteration, ants, eta=None, threads=None,
              want_slots=False, want_probs=False):
    """Build the tours of `ants` (list of ant indices).  Returns a dict with
    tours int32 [A][n], lengths int64 [A], fallbacks int64 [A] and optionally
    slots int8 [A][n] (-1 = fallback) and probs float64 [A][n]."""
    xy = _xy(xy)
    n = len(xy)
    nn = np.ascontiguousarray(nn, np.int32)
    nnd = np.ascontiguousarray(nnd, np.int32)
    tau = np.ascontiguousarray(tau, np.float32)
    eta = None if eta is None else np.ascontiguousarray(eta, np.float64)
    k = nn.shape[1]
    ants = np.ascontiguousarray(ants, np.int64)
    A = len(ants)
    tours = np.empty((A, n), np.int32)
    lengths = np.empty(A, np.int64)
    fb = np.empty(A, np.int64)
    slots = np.empty((A, n), np.int8) if want_slots else None
    probs = np.empty((A, n), np.float64) if want_probs else None
    lib().oracle_construct(n, k, _p(xy), _p(nn), _p(nnd), _p(tau), _p(eta), float(alpha),
                           float(beta), int(seed), int(iteration), _p(ants), A, _p(tours),
                           _p(lengths), _p(slots), _p(probs), _p(fb), _threads(threads))
    out = dict(tours=tours, lengths=lengths, fallbacks=fb)
    if want_slots:
        out["slots"] = slots
    if want_probs:
        out["probs"] = probs
    return out


REPLAY_FIELDS = ("steps", "fallbacks", "near_boundary_mismatch", "hard_mismatch",
                 "fallback_mismatch", "invalid", "near_boundary")


def replay(xy, nn, nnd, tau, alpha, beta, seed, iteration, ant, tour, eta=None,
           boundary_eps=1e-6, sweep=None):
    """Teacher-forced replay of one tour.  Returns (counts dict, prob float64 [n]).
    sweep: None (fallback moves checked by the O(n) brute force) or the
    x_sweep_index of xy (checked by the sweep along x, which gives the same city)."""
    xy = _xy(xy)
    n = len(xy)
    nn = np.ascontiguousarray(nn, np.int32)
    nnd = np.ascontiguousarray(nnd, np.int32)
    tau = np.ascontiguousarray(tau, np.float32)
    eta = None if eta is None else np.ascontiguousarray(eta, np.float64)
    tour = np.ascontiguousarray(tour, np.int32)
    prob = np.zeros(n, np.float64)
    out = np.zeros(8, np.int64)
    order, pos = (None, None) if sweep is None else sweep
    lib().oracle_replay(n, nn.shape[1], _p(xy), _p(nn), _p(nnd), _p(tau), _p(eta), float(alpha),
                        float(beta), int(seed), int(iteration), int(ant), _p(tour),
                        float(boundary_eps), _p(order), _p(pos), _p(prob), _p(out))
    return {f: int(out[i]) for i, f in enumerate(REPLAY_FIELDS)}, prob


# ---------------------------------------------------------------- PartialACO
def p_threshold(p: float) -> int:
    """Threshold P = round(p 2^32) of the partial-modification draw (x1 < P)."""
    return int(min(max(round(float(p) * 2.0**32), 0), 2**32))


def partial_plan(seed, iteration, ant, n, p, max_modify):
    """(start position, partial?, cities rebuilt) of one ant (Section 3.1, Algorithm 1)."""
    s, r = C.c_int64(0), C.c_int64(0)
    part = C.c_int(0)
    lib().oracle_partial_plan(int(seed), int(iteration), int(ant), int(n), p_threshold(p),
                              int(max_modify), C.byref(s), C.byref(part), C.byref(r))
    return int(s.value), bool(part.value), int(r.value)


SAMPLER_ROULETTE = 0      # Eq. 1
SAMPLER_INDEPENDENT = 1   # Independent Roulette (Section 3)


def construct_partial(xy, nn, nnd, tau, alpha, beta, seed, iteration, ants, lbest, p, max_modify,
                      eta=None, sampler=SAMPLER_ROULETTE):
    """PartialACO construction of the listed ants; lbest [len(ants)][n] are their local bests
    (p = 0: full tours).  Returns dict(tours, lengths, slots, probs)."""
    xy = _xy(xy)
    n = len(xy)
    nn = np.ascontiguousarray(nn, np.int32)
    nnd = np.ascontiguousarray(nnd, np.int32)
    tau = np.ascontiguousarray(tau, np.float32)
    eta = None if eta is None else np.ascontiguousarray(eta, np.float64)
    ants = np.ascontiguousarray(ants, np.int64)
    lbest = np.ascontiguousarray(lbest, np.int32)
    A = len(ants)
    tours = np.empty((A, n), np.int32)
    lengths = np.empty(A, np.int64)
    slots = np.empty((A, n), np.int8)
    probs = np.empty((A, n), np.float64)
    lib().oracle_construct_partial(n, nn.shape[1], _p(xy), _p(nn), _p(nnd), _p(tau), _p(eta),
                                   float(alpha), float(beta), int(seed), int(iteration), _p(ants),
                                   A, _p(lbest), p_threshold(p), int(max_modify), int(sampler),
                                   _p(tours), _p(lengths), _p(slots), _p(probs))
    return dict(tours=tours, lengths=lengths, slots=slots, probs=probs)


def replay_partial(xy, nn, nnd, tau, alpha, beta, seed, iteration, ant, lbest, p, max_modify,
                   tour, eta=None, boundary_eps=1e-6, sampler=SAMPLER_ROULETTE):
    """Teacher-forced replay of a PartialACO tour.  Returns (counts dict with 'kept', prob)."""
    xy = _xy(xy)
    n = len(xy)
    nn = np.ascontiguousarray(nn, np.int32)
    nnd = np.ascontiguousarray(nnd, np.int32)
    tau = np.ascontiguousarray(tau, np.float32)
    eta = None if eta is None else np.ascontiguousarray(eta, np.float64)
    lbest = np.ascontiguousarray(lbest, np.int32)
    tour = np.ascontiguousarray(tour, np.int32)
    prob = np.zeros(n, np.float64)
    out = np.zeros(8, np.int64)
    lib().oracle_replay_partial(n, nn.shape[1], _p(xy), _p(nn), _p(nnd), _p(tau), _p(eta),
                                float(alpha), float(beta), int(seed), int(iteration), int(ant),
                                _p(lbest), p_threshold(p), int(max_modify), int(sampler),
                                _p(tour), float(boundary_eps), _p(prob), _p(out))
    res = {f: int(out[i]) for i, f in enumerate(REPLAY_FIELDS)}
    res["kept"] = int(out[7])
    return res, prob


# ---------------------------------------------------------------- windowed 2-opt
def two_opt_selected(seed, iteration, ant, p) -> bool:
    """Does the ant's tour get 2-opt this iteration (word 3 of block (0, ant, iteration, 0)
    below round(p 2^32))?"""
    return bool(lib().oracle_two_opt_selected(int(seed), int(iteration), int(ant),
                                               p_threshold(p)))


def two_opt_best(xy, tour, window):
    """Best improving move (gain < 0, ties to the smaller offset) of every position:
    (gain[n], offset[n]); offset 0 where no move improves."""
    xy = _xy(xy)
    n = len(xy)
    t = np.ascontiguousarray(tour, np.int32)
    g = np.empty(n, np.int64)
    o = np.empty(n, np.int64)
    lib().oracle_two_opt_best(_p(xy), n, _p(t), int(window), _p(g), _p(o))
    return g, o


def two_opt(xy, tour, window, max_rounds=0):
    """Windowed 2-opt of one tour (Sections 4-5), by rounds of non-overlapping best moves.
    Returns (new tour, dict(rounds, moves, gain, converged))."""
    xy = _xy(xy)
    n = len(xy)
    t = np.array(tour, np.int32)
    mv, gn = C.c_int64(0), C.c_int64(0)
    conv = C.c_int(0)
    r = lib().oracle_two_opt(_p(xy), n, _p(t), int(window), int(max_rounds), C.byref(mv),
                             C.byref(gn), C.byref(conv))
    return t, dict(rounds=int(r), moves=int(mv.value), gain=int(gn.value),
                   converged=bool(conv.value))


def pheromone_local_best(nn, lbest, lbest_len, tau_base, delta, shift=32):
    """Pheromone from the local best tours (P-ACO variant, Section 3).
    Returns (tau float32 [n][k], q int64 [m])."""
    nn = np.ascontiguousarray(nn, np.int32)
    lbest = np.ascontiguousarray(lbest, np.int32)
    lbest_len = np.ascontiguousarray(lbest_len, np.int64)
    n, k = nn.shape
    tau = np.empty((n, k), np.float32)
    q = np.empty(len(lbest_len), np.int64)
    lib().oracle_pheromone_local_best(n, k, _p(nn), len(lbest_len), _p(lbest), _p(lbest_len),
                                      float(tau_base), float(delta), int(shift), _p(tau), _p(q))
    return tau, q


def update_local_best(lbest, lbest_len, tours, lengths):
    """Algorithm 1: an ant's local best is replaced only by a strictly shorter tour."""
    lbest = np.array(lbest, np.int32, copy=True)
    lbest_len = np.array(lbest_len, np.int64, copy=True)
    better = np.asarray(lengths) < lbest_len
    lbest[better] = np.asarray(tours)[better]
    lbest_len[better] = np.asarray(lengths)[better]
    return lbest, lbest_len


# ---------------------------------------------------------------- update
def deposit(nn, tours, lengths, shift=32, threads=None) -> np.ndarray:
    nn = np.ascontiguousarray(nn, np.int32)
    tours = np.ascontiguousarray(tours, np.int32)
    lengths = np.ascontiguousarray(lengths, np.int64)
    n, k = nn.shape
    acc = np.empty((n, k), np.int64)
    lib().oracle_deposit(n, k, _p(nn), tours.shape[0], _p(tours), _p(lengths), int(shift), _p(acc),
                         _update_threads(threads, tours.shape[0]))
    return acc


def _update_threads(threads, m) -> int:
    """Threads for the deposit: one for small colonies, else up to 16."""
    if threads:
        return int(threads)
    return 1 if m < 64 else min(16, os.cpu_count() or 1)


def update(nn, tau, tours, lengths, rho, shift=32, threads=None) -> np.ndarray:
    """Return the pheromone after evaporation and deposit (input left untouched)."""
    nn = np.ascontiguousarray(nn, np.int32)
    t = np.array(tau, dtype=np.float32, copy=True, order="C")
    tours = np.ascontiguousarray(tours, np.int32)
    lengths = np.ascontiguousarray(lengths, np.int64)
    n, k = nn.shape
    lib().oracle_update(n, k, _p(nn), _p(t), tours.shape[0], _p(tours), _p(lengths), float(rho),
                        int(shift), _update_threads(threads, tours.shape[0]))
    return t


# ---------------------------------------------------------------- whole loop
def run(xy, m, k, alpha, beta, rho, iterations, seed, shift=32, threads=None):
    """Full run on one instance.  Returns dict(best_tour, best_len, iter_best, tau)."""
    xy = _xy(xy)
    n = len(xy)
    best_tour = np.empty(n, np.int32)
    best_len = np.zeros(1, np.int64)
    iter_best = np.zeros(max(iterations, 1), np.int64)
    tau = np.empty((n, k), np.float32)
    rc = lib().oracle_run(n, k, _p(xy), int(m), float(alpha), float(beta), float(rho),
                          int(iterations), int(seed), int(shift), _threads(threads), _p(best_tour),
                          _p(best_len), _p(iter_best), _p(tau))
    if rc != 0:
        raise ValueError(f"oracle_run failed with code {rc}")
    return dict(best_tour=best_tour, best_len=int(best_len[0]), iter_best=iter_best[:iterations],
                tau=tau)
