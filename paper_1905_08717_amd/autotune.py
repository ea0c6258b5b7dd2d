"""Launch-configuration tuner: picks the grid caps of a batch context by
measuring macro steps of the actual workload.

The knobs (``mr_set_launch``) are the most workgroups given to the
list-driven kernels, to the interface-leaf stage launches and to the list
compaction, and the block-to-level schedule of the bulk stage kernel (one
launch over all levels of a stage, or one per level).  They change no result -- every kernel loops over whatever its
grid does not cover -- only how the work is spread over the 256 compute
units: a grid just above the number of resident workgroups leaves a second,
mostly idle round; a much larger one adds per-workgroup set-up.  The right
value depends on the kernels' register use (resident waves) and on the
workload, so it is measured, not derived.

Search: coordinate descent, one knob at a time over its candidates with the
others fixed, two passes.  Each trial reloads the same initial data, runs
``warmup`` macro steps (the first one also captures the macro-step graph)
and times ``steps`` more on the context's stream.

The chosen settings are kept in ``tuned_launch.json`` beside this file,
one record per workload key, so that a run can use a measured setting
without searching again (``record`` / ``lookup``).
"""
from __future__ import annotations

import json
import os
import time

CANDIDATES = {
    "list_grid": (128, 256, 512, 1024, 1536, 1792, 2048, 3072, 4096, 6144, 8192),
    "iface_grid": (64, 128, 256, 512, 1024, 2048),
    "comp_grid": (256, 512, 1024, 2048, 4096, 8192, 16384),
    # block-to-level schedule of the bulk stage kernel: one launch over all
    # levels of a stage, or one per level
    "bulk_levels": (1, 2),
}


def time_config(solver, q0, dt, knobs: dict, warmup: int, steps: int) -> float:
    """Seconds per macro step of `solver` with the launch knobs `knobs`,
    starting from `q0` (device tensor or array) each time; dt: dt_L, one
    value or one per instance."""
    import torch

    solver.set_launch(**knobs)
    solver.load_finest(q0)
    for _ in range(warmup):
        solver.lt_step(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.lt_step(dt)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def tune(solver, q0, dt, warmup: int = 1, steps: int = 2, passes: int = 2, candidates=None, log=None,
         margin: float = 0.02):
    """Coordinate descent over the launch knobs of `solver`; a candidate
    replaces the incumbent only when it is faster by more than `margin`
    (so timing noise does not flip the choice).  Leaves the best setting
    applied and returns {"best": knobs, "seconds_per_step": t, "default": t0,
    "trials": [...]}."""
    cand = dict(CANDIDATES if candidates is None else candidates)
    best = dict(solver.get_launch())
    trials = []
    t_best = time_config(solver, q0, dt, best, warmup, steps)
    t_default = t_best
    trials.append((dict(best), t_best))
    for _ in range(passes):
        improved = False
        for name, values in cand.items():
            for v in values:
                if v == best[name]:
                    continue
                knobs = dict(best, **{name: v})
                t = time_config(solver, q0, dt, knobs, warmup, steps)
                trials.append((dict(knobs), t))
                if log:
                    log(f"[tune] {knobs} {1e3 * t:.2f} ms/step")
                if t < t_best * (1.0 - margin):
                    best, t_best, improved = knobs, t, True
        if not improved:
            break
    solver.set_launch(**best)
    return {"best": best, "seconds_per_step": t_best, "default": t_default,
            "trials": [{"knobs": k, "seconds_per_step": t} for k, t in trials]}


RECORD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_launch.json")


def lookup(key: str, path: str = RECORD_PATH):
    """The stored launch knobs of workload `key`, or None."""
    try:
        with open(path) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    # records taken before a knob existed keep its default (omitted here)
    return {k: int(rec[k]) for k in CANDIDATES if k in rec}


def record(key: str, result: dict, note: str, path: str = RECORD_PATH):
    """Store the outcome of `tune` for workload `key`."""
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data[key] = dict(result["best"], ms_per_step=round(1e3 * result["seconds_per_step"], 3),
                     ms_per_step_default=round(1e3 * result["default"], 3), trials=len(result["trials"]),
                     how=note)
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")


def nagumo_key(L: int, batch: int) -> str:
    return f"nagumo2d_L{L}_b{batch}"


def euler3d_key(L: int) -> str:
    return f"euler3d_L{L}_b1"


def main():
    import argparse
    import sys

    import numpy as np
    import torch

    from paper_1905_08717_amd import mrlt
    from paper_1905_08717_amd import workloads as W

    ap = argparse.ArgumentParser(description="tune the launch knobs for a batch of 2D Nagumo fronts, "
                                             "or for the 3D Euler spherical Riemann problem")
    ap.add_argument("--workload", choices=["nagumo2d", "euler3d"], default="nagumo2d")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--L", type=int, default=0, help="finest level (default 9 for nagumo2d, 7 for euler3d)")
    ap.add_argument("--out", default="")
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--record", action="store_true", help="store the result in tuned_launch.json")
    ap.add_argument("--record-path", default=RECORD_PATH)
    args = ap.parse_args()
    if args.workload == "euler3d":
        # one solve; the step of the first macro step (CFL from the initial
        # wave speeds) is held for every trial
        L = args.L or 7
        cfg = W.euler_3d(L=L)
        q0 = torch.from_numpy(W.euler_sphere(L)[None]).to("cuda")
        s = mrlt.Solver(cfg)
        s.load_finest(q0)
        dt = W.euler_dt(cfg, s.max_wavespeed()[0], 0.0)
        key = euler3d_key(L)
    else:
        L = args.L or 9
        cfg = W.nagumo_2d(L=L)
        q0 = torch.from_numpy(np.stack([W.nagumo_front(L, W.SEED + i) for i in range(args.batch)])).to("cuda")
        s = mrlt.Solver(cfg, n_inst=args.batch)
        dt = W.nagumo_dt(cfg)
        key = nagumo_key(L, args.batch)
    r = tune(s, q0, dt, steps=args.steps, passes=args.passes,
             log=lambda m: print(m, file=sys.stderr, flush=True))
    if args.record:
        record(key, r,
               f"coordinate descent, {args.passes} passes, 1 warm-up and {args.steps} timed macro steps per trial",
               path=args.record_path)
    text = json.dumps(r, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
