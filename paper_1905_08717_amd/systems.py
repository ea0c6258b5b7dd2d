"""Systems forms on one GPU: many independent MRLT/NERK3 solves.

* Batched: uneven solves (different finest level, threshold, initial data)
  advanced together; solves of one problem class (PDE, dimension, finest
  level) share a batch context, so every kernel launch of a macro step
  serves all of them.  Each solve keeps its own CFL step and stops at its
  own final time; a finished solve's slot is freed (all cells absent), so it
  drops out of every kernel's work.
* Served: requests arrive over time (Poisson); a request is admitted into a
  free slot of its class as soon as one is free and the class's device
  memory budget allows, is advanced one macro step at a time together with
  whatever else is resident, and its result is read back when it reaches its
  final time.  Latency = arrival to result ready.

All numerical work runs in the HIP library through the C ABI; this module
only schedules.
"""
from __future__ import annotations

import dataclasses
import heapq
import math
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
    return (cfg["pde"], cfg["dim"], cfg["L"], cfg.get("l0", 2))


def bytes_per_instance(cfg: dict) -> int:
    """Device bytes of one slot: cell tables of all levels (status, scratch,
    ghost flag, three int lists, nine FP64 slots of m fields) and the flux
    registers of the levels below L."""
    d, L, l0 = cfg["dim"], cfg["L"], cfg.get("l0", 2)
    m = W.ncomp(cfg)
    cells = sum(1 << (d * lev) for lev in range(l0, L + 1))
    coarse = sum(1 << (d * lev) for lev in range(l0, L))
    regs = coarse * 2 * d * (1 + (1 << (d - 1))) * m * 8
    return cells * (3 + 12 + 9 * m * 8) + regs


def step_dt(cfg: dict, ws: float, t: float, t_final: float) -> float:
    """Finest-level step of one solve for its next macro step: CFL sigma on
    the finest level (advective and diffusive limits), cut so that the last
    macro step ends exactly at t_final."""
    it = W.macro_iters(cfg)
    dx = (cfg.get("hi", [1.0] * 3)[0] - cfg.get("lo", [0.0] * 3)[0]) / (1 << cfg["L"])
    sigma = cfg.get("cfl", 0.5)
    rate = ws / dx
    if cfg["pde"] in ("burgers", "nagumo", "linear"):
        rate += 2 * cfg["dim"] * cfg.get("nu", 0.0) / dx ** 2
    if cfg["pde"] == "nagumo":
        rate += 0.8 * cfg.get("k_react", 0.0)
    dt = sigma / rate if rate > 0 else (t_final - t) / it
    return min(dt, (t_final - t) / it)


class SlotPool:
    """One batch context with `slots` instances for one problem class."""

    def __init__(self, cfg: dict, slots: int, eps: List[float] = None):
        self.cfg = dict(cfg)
        self.slots = slots
        self.solver = mrlt.Solver(cfg, n_inst=slots, eps=eps or [cfg.get("eps", 1e-3)] * slots)
        self.req: List[Optional[Request]] = [None] * slots
        self.failed: List[Request] = []
        self.t = np.zeros(slots)

    def free_slots(self) -> List[int]:
        return [i for i, r in enumerate(self.req) if r is None]

    def active(self) -> int:
        return sum(r is not None for r in self.req)

    def admit(self, r: Request, slot: int):
        self.solver.set_eps(slot, r.eps)
        self.solver.load_finest_inst(slot, r.q0)
        self.req[slot] = r
        self.t[slot] = 0.0

    def load_all(self, reqs: List[Request]):
        """Admit a full batch at once (one load for all slots)."""
        assert len(reqs) == self.slots
        q = np.stack([r.q0 for r in reqs])
        for i, r in enumerate(reqs):
            self.solver.set_eps(i, r.eps)
        self.solver.load_finest(q)
        self.req = list(reqs)
        self.t[:] = 0.0

    def step(self) -> int:
        """One macro step of every resident solve; returns the number stepped."""
        n = self.active()
        if n == 0:
            return 0
        ws = self.solver.max_wavespeed()
        dts = np.ones(self.slots)
        for i, r in enumerate(self.req):
            if r is not None:
                dts[i] = step_dt(self.cfg, ws[i], self.t[i], r.t_final)
        rc = self.solver.lt_step_rc_batch(dts)
        if rc in (mrlt.ENONFINITE, mrlt.ESTATE):
            # a failing request fails alone: retire it, keep the others
            for i, r in enumerate(self.req):
                if r is not None and self.solver.instance_flags(i):
                    r.failed = True
                    r.t_final = self.t[i]
            for i, r in enumerate(self.req):
                if r is not None and r.failed:
                    self.solver.clear_instance(i)
                    self.failed.append(r)
                    self.req[i] = None
        elif rc != mrlt.OK:
            raise mrlt.MrError(rc, self.solver.last_error())
        it = W.macro_iters(self.cfg)
        for i, r in enumerate(self.req):
            if r is not None:
                self.t[i] += it * dts[i]
                r.macro_steps += 1
        return n

    def poll(self, now: float, keep_result: bool = True) -> List[Request]:
        """Finished solves: read their leaves, free their slots."""
        out = []
        for i, r in enumerate(self.req):
            if r is not None and self.t[i] >= r.t_final * (1 - 1e-12):
                if keep_result:
                    r.result = self.solver.get_leaves(i)
                r.done_at = now
                self.solver.clear_instance(i)
                self.req[i] = None
                out.append(r)
        return out


class _Progress:
    """A line on stderr every `every` seconds (long runs stay visibly alive)."""

    def __init__(self, what: str, every: float = 10.0):
        self.what, self.every = what, every
        self.t0 = self.last = time.perf_counter()

    def __call__(self, msg: str):
        now = time.perf_counter()
        if now - self.last >= self.every:
            self.last = now
            print(f"[{self.what}] {now - self.t0:.1f} s: {msg}", file=sys.stderr, flush=True)


def run_batched(reqs: List[Request]) -> Dict:
    """Advance all requests to completion, batched by problem class."""
    groups: Dict[tuple, List[Request]] = {}
    for r in reqs:
        groups.setdefault(class_key(r.cfg), []).append(r)
    t0 = time.perf_counter()
    pools = []
    for key, rs in groups.items():
        p = SlotPool(rs[0].cfg, len(rs), eps=[r.eps for r in rs])
        p.load_all(rs)
        pools.append(p)
    done = 0
    steps = 0
    prog = _Progress("batched")
    # a request that fails (non-finite state) is retired alone; it counts as
    # ended but not as solved
    while done + sum(len(p.failed) for p in pools) < len(reqs):
        for p in pools:
            steps += p.step()
            done += len(p.poll(time.perf_counter() - t0))
        prog(f"{done}/{len(reqs)} solves done, {steps} slot macro steps")
    el = time.perf_counter() - t0
    failed = sum(len(p.failed) for p in pools)
    return {"seconds": el, "solves": done, "failed": failed, "solves_per_s": done / el,
            "slot_macro_steps": steps}


def run_one_at_a_time(reqs: List[Request]) -> Dict:
    """The plain GPU form: every request alone in a batch of one."""
    pools: Dict[tuple, SlotPool] = {}
    t0 = time.perf_counter()
    prog = _Progress("one-at-a-time")
    for k, r in enumerate(reqs):
        key = class_key(r.cfg)
        if key not in pools:
            pools[key] = SlotPool(r.cfg, 1, eps=[r.eps])
        p = pools[key]
        p.admit(r, 0)
        while p.active():
            p.step()
            p.poll(time.perf_counter() - t0)
            prog(f"solve {k + 1}/{len(reqs)}")
    el = time.perf_counter() - t0
    failed = sum(len(p.failed) for p in pools.values())
    done = len(reqs) - failed
    return {"seconds": el, "solves": done, "failed": failed, "solves_per_s": done / el}


def serve(reqs: List[Request], hbm_budget: float, max_slots: int = 64) -> Dict:
    """Continuous batching: admit requests as they arrive and as slots and the
    memory budget allow, step every class with resident solves, retire
    finished ones.  Arrival times are in seconds from the start."""
    pending = sorted(reqs, key=lambda r: r.arrival)
    queue: List[Request] = []
    pools: Dict[tuple, SlotPool] = {}
    used = 0.0
    stalls = 0
    t0 = time.perf_counter()
    finished: List[Request] = []
    nxt = 0
    prog = _Progress("served")
    while len(finished) + sum(len(p.failed) for p in pools.values()) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(pending) and pending[nxt].arrival <= now:
            queue.append(pending[nxt])
            nxt += 1
        # admission, first come first served, per class
        still = []
        for r in queue:
            key = class_key(r.cfg)
            if key not in pools:
                need = bytes_per_instance(r.cfg) * max_slots
                if used + need > hbm_budget:
                    still.append(r)
                    stalls += 1
                    continue
                pools[key] = SlotPool(r.cfg, max_slots)
                used += need
            p = pools[key]
            free = p.free_slots()
            if not free:
                still.append(r)
                stalls += 1
                continue
            p.admit(r, free[0])
        queue = still
        stepped = 0
        for p in pools.values():
            stepped += p.step()
            for r in p.poll(time.perf_counter() - t0, keep_result=False):
                finished.append(r)
        prog(f"{len(finished)}/{len(reqs)} finished, {len(queue)} queued, {nxt} arrived")
        if stepped == 0 and nxt < len(pending) and not queue:
            wait = pending[nxt].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    makespan = time.perf_counter() - t0
    lat = np.array([r.done_at - r.arrival for r in finished])
    failed = sum(len(p.failed) for p in pools.values())
    return {"requests": len(reqs), "failed": failed, "makespan_s": makespan,
            "solves_per_s": len(finished) / makespan,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "admission_stalls": stalls, "classes": len(pools), "hbm_reserved_bytes": used}


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
