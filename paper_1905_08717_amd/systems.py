"""Systems forms on one GPU: many independent MRLT/NERK3 solves, driven
through the library's scheduler (mr_batch_* of the C ABI).

* Batched: uneven solves (different finest level, threshold, initial data)
  in one class per scheme, whose context has the largest finest level: every
  kernel launch of a macro step serves all of them.  Each solve keeps its
  own CFL step and stops at its own final time.
* Served: requests arrive over time (Poisson) and are admitted as slots and
  device memory free up; classes (one per scheme and finest level) step on
  their own streams; results are read back as solves finish.
* One at a time: the plain form, every request alone in a context of its own
  finest level.

All numerical work and the scheduling of slots, steps and memory run in the
native library; this module only feeds requests and reads results.
"""
from __future__ import annotations

import dataclasses
import sys
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import mrlt
from . import workloads as W


@dataclasses.dataclass
class Request:
    rid: int
    cfg: dict                 # problem class + parameters (dim, L, pde, ...)
    eps: float
    q0: np.ndarray            # (m, 2^{dL}) finest-level averages
    t_final: float
    arrival: float = 0.0      # seconds after the start of the run
    done_at: Optional[float] = None
    result: Optional[Tuple[np.ndarray, np.ndarray]] = None
    macro_steps: int = 0
    failed: bool = False


def class_key(cfg: dict) -> tuple:
    """Solves that may share a context: same PDE, dimension, coarsest level
    and scheme parameters (the finest level may differ)."""
    skip = ("L", "eps", "name", "t_final")
    return tuple(sorted((k, repr(v)) for k, v in cfg.items() if k not in skip))


def _m(cfg: dict) -> int:
    return W.ncomp(cfg)


def _progress(what: str, every: float = 10.0):
    """A line on stderr every `every` seconds (long runs stay visibly alive)."""
    state = {"t0": time.perf_counter(), "last": time.perf_counter()}

    def tick(msg: str):
        now = time.perf_counter()
        if now - state["last"] >= every:
            state["last"] = now
            print(f"[{what}] {now - state['t0']:.1f} s: {msg}", file=sys.stderr, flush=True)
    return tick


def _drain(b: mrlt.Batch, by_slot: Dict[int, Request], now: float) -> Tuple[List[Request], List[Request]]:
    """Finished and failed solves of the last steps: results read, slots freed."""
    done, failed = [], []
    for slot in b.poll():
        r = by_slot.pop(slot)
        info = b.slot_info(slot)
        r.macro_steps = info["macro_steps"]
        if info["state"] == mrlt.SLOT_DONE:
            r.result = b.get_leaves(slot, _m(r.cfg))
            r.done_at = now
            done.append(r)
        else:
            r.failed = True
            failed.append(r)
        b.release(slot)
    return done, failed


def run_batched(reqs: List[Request], hbm_budget: int = 200 * 2 ** 30) -> Dict:
    """All requests in as few contexts as their schemes allow: one class per
    scheme with the largest finest level of its requests and a slot for each,
    so solves of uneven finest level share every launch.  Time from the
    first admission to the last result."""
    groups: Dict[tuple, List[Request]] = {}
    for r in reqs:
        groups.setdefault(class_key(r.cfg), []).append(r)
    classes = [(rs[0].cfg, max(r.cfg["L"] for r in rs), len(rs)) for rs in groups.values()]
    b = mrlt.Batch(classes, hbm_budget)
    t0 = time.perf_counter()
    by_slot: Dict[int, Request] = {}
    for r in reqs:
        slot = b.admit(r.cfg, r.cfg["L"], r.eps, r.t_final, r.q0, cfl=r.cfg.get("cfl", 0.5))
        if slot is None:
            raise RuntimeError("batched form: the requests do not fit the HBM budget")
        by_slot[slot] = r
    done, failed, steps = 0, 0, 0
    tick = _progress("batched")
    while by_slot:
        b.step()
        steps += 1
        d, f = _drain(b, by_slot, time.perf_counter() - t0)
        done += len(d)
        failed += len(f)
        tick(f"{done}/{len(reqs)} solves done, {steps} macro steps")
    el = time.perf_counter() - t0
    fp = b.footprint()
    b.close()
    return {"seconds": el, "solves": done, "failed": failed, "solves_per_s": done / el,
            "macro_steps": steps, "hbm_bytes": fp}


def run_one_at_a_time(reqs: List[Request], hbm_budget: int = 200 * 2 ** 30) -> Dict:
    """The plain GPU form: every request alone, one after another, in a
    context of its own finest level (one per class and level, reused)."""
    keys = []
    for r in reqs:
        k = (class_key(r.cfg), r.cfg["L"])
        if k not in keys:
            keys.append(k)
    first = {}
    for r in reqs:
        first.setdefault((class_key(r.cfg), r.cfg["L"]), r.cfg)
    b = mrlt.Batch([(first[k], k[1], 1) for k in keys], hbm_budget)
    t0 = time.perf_counter()
    done, failed = 0, 0
    tick = _progress("one-at-a-time")
    for j, r in enumerate(reqs):
        slot = b.admit(r.cfg, r.cfg["L"], r.eps, r.t_final, r.q0, cfl=r.cfg.get("cfl", 0.5))
        by_slot = {slot: r}
        while by_slot:
            b.step()
            d, f = _drain(b, by_slot, time.perf_counter() - t0)
            done += len(d)
            failed += len(f)
        tick(f"solve {j + 1}/{len(reqs)}")
    el = time.perf_counter() - t0
    b.close()
    return {"seconds": el, "solves": done, "failed": failed, "solves_per_s": done / el}


def serve(reqs: List[Request], hbm_budget: float, slots: int = 16) -> Dict:
    """Continuous batching: requests join the run as they arrive and as
    slots and device memory allow (the library's admission), every class
    with running solves advances one macro step per round on its own stream,
    and finished solves are read back and their slots freed at once.
    Classes: one per scheme and finest level, `slots` slots each.  Arrival
    times are seconds from the start; latency = arrival to result."""
    first: Dict[tuple, dict] = {}
    for r in reqs:
        first.setdefault((class_key(r.cfg), r.cfg["L"]), r.cfg)
    keys = sorted(first, key=lambda k: (k[1], str(k[0])))
    b = mrlt.Batch([(first[k], k[1], slots) for k in keys], int(hbm_budget))
    pending = sorted(reqs, key=lambda r: r.arrival)
    queue: List[Request] = []
    by_slot: Dict[int, Request] = {}
    finished: List[Request] = []
    failed: List[Request] = []
    stalls = 0
    peak = 0
    nxt = 0
    t0 = time.perf_counter()
    tick = _progress("served")
    while len(finished) + len(failed) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(pending) and pending[nxt].arrival <= now:
            queue.append(pending[nxt])
            nxt += 1
        still = []
        for r in queue:
            slot = b.admit(r.cfg, r.cfg["L"], r.eps, r.t_final, r.q0, cfl=r.cfg.get("cfl", 0.5))
            if slot is None:
                still.append(r)
                stalls += 1
            else:
                by_slot[slot] = r
        queue = still
        peak = max(peak, b.footprint())
        if by_slot:
            b.step()
            d, f = _drain(b, by_slot, time.perf_counter() - t0)
            finished += d
            failed += f
        elif nxt < len(pending):
            wait = pending[nxt].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
        tick(f"{len(finished)}/{len(reqs)} finished, {len(queue)} queued, {len(by_slot)} running, {nxt} arrived")
    makespan = time.perf_counter() - t0
    b.close()
    lat = np.array([r.done_at - r.arrival for r in finished])
    return {"requests": len(reqs), "failed": len(failed), "makespan_s": makespan,
            "solves_per_s": len(finished) / makespan,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "admission_stalls": stalls, "classes": len(keys), "hbm_peak_bytes": peak}


# ---------------------------------------------------------------------------
# workloads of the two systems forms


def batched_euler_requests(n: int = 256, seed: int = W.SEED) -> List[Request]:
    """Four-quadrant 2D Euler Riemann problems: seeded states, finest level
    from {7, 8, 9}, threshold from {1e-2, 1e-3, 1e-4}, t_final = 0.25."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(rng.choice([7, 8, 9]))
        eps = float(rng.choice([1e-2, 1e-3, 1e-4]))
        cfg = W.euler_2d(L=L, eps=eps)
        out.append(Request(i, cfg, eps, W.euler_quadrants_seeded(L, seed + i), 0.25))
    return out


def served_requests(n: int = 1000, rate: float = 200.0, seed: int = W.SEED + 1_000_000,
                    burgers_levels=(10, 11, 12, 13, 14), rd_levels=(7, 8, 9)) -> List[Request]:
    """Poisson arrivals (mean `rate` per s), half 1D viscous Burgers (sine or
    four-mode random-phase data, t_final 0.5), half 2D Nagumo fronts
    (t_final 0.01); eps log-uniform in [1e-4, 1e-2]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        eps = float(10 ** rng.uniform(-4, -2))
        if rng.random() < 0.5:
            L = int(rng.choice(burgers_levels))
            cfg = W.burgers_1d(L=L, eps=eps)
            if rng.random() < 0.5:
                q0 = W.burgers_sine(L, phase=float(rng.uniform(0, 1)))
            else:
                q0 = W.burgers_modes(L, int(rng.integers(1 << 30)))
            out.append(Request(i, cfg, eps, q0, 0.5, arrival=t))
        else:
            L = int(rng.choice(rd_levels))
            cfg = W.nagumo_2d(L=L, eps=eps)
            out.append(Request(i, cfg, eps, W.nagumo_front(L, int(rng.integers(1 << 30))), 0.01, arrival=t))
    return out
