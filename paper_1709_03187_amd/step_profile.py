"""Where a construction step's time goes, from the step profile build.

    python -m paper_1709_03187_amd.build --step-profile
    python -m paper_1709_03187_amd.step_profile [--iterations 6] [--out FILE]

Runs the n = 200,000 clustered workload (m = 1,024, k = 16) on
libaco_step_profile.so, whose construction kernels stamp the shader clock at
five points of every step (the current row has arrived; its visited test is
known; on roulette steps, the running sums' total is known; the next city is
known; the end of the step) and keep per-ant sums.  The last iteration's
counters are summarised per ant-step: row wait, the visited test, the
decision by path (the roulette's scan and its draw and pick,
nearest-unvisited fallback split by duration), the rest of the step, and the
work between blocks of 64 steps; the iteration before is run with the grid
searches' pass and point counters on (their atomics would distort the
clock).  The tours are those of the
library (the stamps change no result); the clock adds a few instructions per
step, so the profiled kernel runs somewhat slower than the library's.
"""
from __future__ import annotations

import argparse
import ctypes as C
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE_LIB = os.path.join(HERE, "libaco_step_profile.so")
FIELDS = ["total", "row_wait", "tail", "block", "decide_roulette", "decide_fallback",
          "decide_ir", "count_roulette", "count_fallback", "count_ir", "steps", "visited",
          "fb_mid_n", "fb_mid_t", "fb_long_n", "fb_long_t", "scan", "spare"]
FB_MID_TICKS, FB_LONG_TICKS = 2000, 6000   # the kernel's duration classes
NFIELDS = 18


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iterations", type=int, default=6)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if not os.path.exists(PROFILE_LIB):
        sys.exit(f"{PROFILE_LIB} is not built: python -m paper_1709_03187_amd.build --step-profile")
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    import paper_1709_03187_amd as aco
    from paper_1709_03187_amd import instances

    aco.LIB_PATH = PROFILE_LIB      # the profile build in place of libaco.so
    L = aco.lib()
    L.aco_step_profile_buffer.restype = None
    L.aco_step_profile_buffer.argtypes = [C.c_void_p]
    L.aco_grid_stats.restype = C.c_int
    L.aco_grid_stats.argtypes = [C.c_void_p, C.c_int]
    grid_stats = (C.c_uint64 * 4)()
    cfg = instances.CONFIGS["c3"]
    xy = instances.make_coords("c3")
    n, m, k = cfg["n"], cfg["m"], cfg["k"]
    col = aco.Colony(xy=xy, k=k, m=m, alpha=cfg["alpha"], beta=cfg["beta"], rho=cfg["rho"],
                     seed=cfg["seed"])
    col.setup()
    prof = torch.zeros((m, NFIELDS), dtype=torch.int64, device="cuda")
    last = args.iterations - 1
    for it in range(args.iterations):
        # grid-search counters on for the iteration before the timed one
        if it == last - 1 or (last == 0 and it == 0):
            torch.cuda.synchronize()
            L.aco_grid_stats(grid_stats, 1)
        if it == last:
            torch.cuda.synchronize()
            if last > 0 and L.aco_grid_stats(grid_stats, 0) != 0:
                sys.exit("reading the grid-search counters failed")
            L.aco_step_profile_buffer(C.c_void_p(prof.data_ptr()))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        col.construct(it)
        e1.record()
        col.update()
        torch.cuda.synchronize()
        print(f"[step profile] iteration {it}: construct {e0.elapsed_time(e1):.2f} ms",
              file=sys.stderr, flush=True)
        if it == last:
            construct_ms = e0.elapsed_time(e1)
    L.aco_step_profile_buffer(None)
    if last == 0 and L.aco_grid_stats(grid_stats, 0) != 0:
        sys.exit("reading the grid-search counters failed")
    gs = [float(v) for v in grid_stats]
    grid_it = last - 1 if last > 0 else 0
    P = prof.cpu().numpy().astype(np.float64)
    steps = P[:, FIELDS.index("steps")]
    total = P[:, 0]
    ticks_per_ms = total.max() / construct_ms
    per_step = {f: float((P[:, i] / steps).mean()) for i, f in enumerate(FIELDS)
                if not f.startswith("count_") and f not in ("steps", "spare")
                and not f.endswith("_n")}
    counts = {f[6:]: float(P[:, FIELDS.index(f)].sum() / steps.sum())
              for f in FIELDS if f.startswith("count_")}
    t_step = per_step["total"]
    rows = [("row wait (end of the previous step until the current row has arrived)",
             per_step["row_wait"]),
            ("visited test of the row's candidates (LDS read, ballot)", per_step["visited"]),
            ("decision: guess load issue and FP64 scan (roulette steps)", per_step["scan"]),
            ("decision: draw and pick (roulette steps)", per_step["decide_roulette"]),
            ("decision: nearest-unvisited fallback (table rows, grid search)",
             per_step["decide_fallback"]),
            ("decision: Independent Roulette", per_step["decide_ir"]),
            ("rest of the step (miss load issue, visited bit, staging)", per_step["tail"]),
            ("between blocks of 64 steps (Philox, stores, tour entries)", per_step["block"])]
    accounted = sum(v for _, v in rows)
    lines = [f"# Construction step profile: n={n:,} clustered, m={m:,}, k={k}, iteration {last}",
             "",
             "Commands (repository root, one MI355X):",
             "",
             "    python -m paper_1709_03187_amd.build --step-profile",
             "    python -m paper_1709_03187_amd.step_profile --iterations "
             f"{args.iterations}" + (f" --out {args.out}" if args.out else ""),
             "",
             f"Profiled construction {construct_ms:.2f} ms; clock ticks of the slowest ant "
             f"{total.max():.4g} ({ticks_per_ms:.4g} ticks per ms); mean "
             f"{t_step:.1f} ticks per ant-step, {1e6 * t_step / ticks_per_ms:.1f} ns.",
             "",
             "| part of a step | ticks per ant-step (mean over ants) | share |",
             "|---|---:|---:|"]
    for label, v in rows:
        lines.append(f"| {label} | {v:.1f} | {v / t_step:.3f} |")
    lines.append(f"| unaccounted (set-up, kept part, the final reduction) | "
                 f"{t_step - accounted:.1f} | {(t_step - accounted) / t_step:.3f} |")
    lines += ["", "Steps by decision path (share of all steps): " +
              ", ".join(f"{f} {v:.4f}" for f, v in counts.items()), ""]
    dec_per = {f: float((P[:, FIELDS.index("decide_" + f)].sum() +
                         (P[:, FIELDS.index("scan")].sum() if f == "roulette" else 0.0)) /
                        max(1.0, P[:, FIELDS.index("count_" + f)].sum()))
               for f in ("roulette", "fallback", "ir")}
    lines.append("Ticks per decision on each path: " +
                 ", ".join(f"{f} {v:.1f}" for f, v in dec_per.items()))
    # fallback decisions by duration: below FB_MID_TICKS (settled by the first
    # table chunk), up to FB_LONG_TICKS (later chunks), above (grid search)
    fb_n = P[:, FIELDS.index("count_fallback")].sum()
    fb_t = P[:, FIELDS.index("decide_fallback")].sum()
    mid_n, mid_t = P[:, FIELDS.index("fb_mid_n")].sum(), P[:, FIELDS.index("fb_mid_t")].sum()
    lng_n, lng_t = P[:, FIELDS.index("fb_long_n")].sum(), P[:, FIELDS.index("fb_long_t")].sum()
    all_steps = steps.sum()
    lines += ["", "Fallback decisions by duration (ticks):", "",
              "| class | share of steps | mean ticks | ticks per ant-step |", "|---|---:|---:|---:|"]
    for label, cn, ct in ((f"< {FB_MID_TICKS}", fb_n - mid_n - lng_n, fb_t - mid_t - lng_t),
                          (f"{FB_MID_TICKS}-{FB_LONG_TICKS}", mid_n, mid_t),
                          (f">= {FB_LONG_TICKS}", lng_n, lng_t)):
        lines.append(f"| {label} | {cn / all_steps:.4f} | {ct / max(1.0, cn):.0f} | "
                     f"{ct / all_steps:.1f} |")
    if gs[0] > 0:
        lines += ["", f"Grid searches (all ants, iteration {grid_it}, counted in a pass the "
                  f"clock profile does not time): {gs[0]:.0f}, "
                  f"{gs[1] / gs[0]:.2f} passes each, {gs[2] / max(1.0, gs[1]):.2f} batches of 64 "
                  f"points per pass, {gs[3] / max(1.0, gs[2]):.1f} points per batch "
                  f"({gs[3] / gs[0]:.0f} points in the searched ranges per search)."]
    text = "\n".join(lines) + "\n"
    print(text)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)


if __name__ == "__main__":
    main()
