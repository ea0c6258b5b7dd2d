#!/usr/bin/env python3
"""Benchmark: leaf cell-updates/s of MRLT/NERK3 macro steps on one MI355X.

Workload: the 2D Nagumo flame-front configuration (512^2 finest cells, L=9,
l0=2, eps=1e-3 with level-dependent thresholds, k=1e3, a=0.2, Neumann unit
square, CFL 0.5, dt_L = 4.76372e-7 so that t=0.01 is 164 macro steps), run
as a batch of B independently seeded fronts advanced by the same launches.
A step is one macro step (2^{L-l0} = 128 fine iterations of every stage
of the method, remesh included) over the whole batch.

value  = leaf-updates (one per leaf per full RK step, counted on the device)
         over the K timed macro steps / wall time, inputs resident in HBM.
roofline = the bulk RK stage kernel (the data-parallel hot path): algorithmic
         bytes 16m / 24m / 24m per leaf and stage (read q^n, write q*; read
         q^n, q*, write q**; read q^n, q**, write q^{n+1}), leaf-stage updates
         counted on the device, over the kernel's HIP-event time.
cpu_baseline = the CPU oracle on one instance of the same workload.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np


def total_updates(s):
    return int(sum(int(s.level_updates(i).sum()) for i in range(s.n_inst)))


def leaf_counts(s):
    tot = np.zeros(25, dtype=np.int64)
    for i in range(s.n_inst):
        tot += np.array(s.stats(i)["leaves"], dtype=np.int64)
    return tot


def stage_traffic(batch, list_grid):
    """HBM bytes per launch of the bulk stage kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, when they were taken on this batch
    size, this grid of the list-driven kernels and the current kernel
    source; otherwise None."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "stage_bulk_traffic.json")
    src = os.path.join(here, "paper_1905_08717_amd", "csrc", "kernels.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256") != digest or rec.get("batch") != batch:
        return None
    if rec.get("launch", {}).get("list_grid") != list_grid:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_oracle_leg(seconds):
    """One timing of the oracle as it is (this process's OpenMP threads): one
    front of the 2D Nagumo configuration, macro steps from t=0 for about
    `seconds` (initial data and the load excluded); prints one JSON line."""
    from oracle import mro
    from paper_1905_08717_amd import workloads as W
    cfg = W.nagumo_2d()
    dt = W.nagumo_dt(cfg)
    o = mro.Oracle(cfg)
    o.load_finest(W.nagumo_front(cfg["L"], W.SEED))
    u0 = o.stats()["leaf_updates"]
    t0 = time.perf_counter()
    nmac = 0
    while True:
        o.lt_step(dt)
        nmac += 1
        el = time.perf_counter() - t0
        if el > seconds or nmac >= 64:
            break
    upd = o.stats()["leaf_updates"] - u0
    print(json.dumps({"leaf_updates_per_s": upd / el, "threads": mro.num_threads(), "macro_steps": nmac,
                      "leaf_updates": upd, "seconds": el}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds, repeats=3):
    """The oracle timed on this host's cores: single-threaded and on every
    core the process may use (OMP_NUM_THREADS as set, else all), each the
    median of `repeats` runs in a fresh process."""
    import statistics
    import subprocess
    here = os.path.abspath(__file__)
    legs = {}
    for name, threads in (("single_thread", "1"), ("all_cores", os.environ.get("OMP_NUM_THREADS", ""))):
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = threads
        else:
            env.pop("OMP_NUM_THREADS", None)
        runs = []
        for _ in range(repeats):
            out = subprocess.run([sys.executable, here, "--mode", "cpu-oracle", "--cpu-seconds", str(seconds)],
                                 env=env, capture_output=True, text=True, check=True)
            runs.append(json.loads(out.stdout.strip().splitlines()[-1]))
            print(f"[bench] cpu oracle {name}: {runs[-1]['leaf_updates_per_s']:.3e} leaf-updates/s", file=sys.stderr,
                  flush=True)
        legs[name] = {"value": statistics.median(r["leaf_updates_per_s"] for r in runs),
                      "runs": [round(r["leaf_updates_per_s"], 1) for r in runs], "threads": runs[0]["threads"]}
    allc = legs["all_cores"]
    return {"value": round(allc["value"], 1), "unit": "leaf-updates/s", "cores": allc["threads"], "kind": "oracle",
            "single_thread": round(legs["single_thread"]["value"], 1),
            "single_thread_runs": legs["single_thread"]["runs"], "all_core_runs": allc["runs"],
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"one front of the same workload (2D Nagumo L=9), macro steps from t=0 for about {seconds} s "
                      f"per run, median of {repeats} runs each single-threaded and on {allc['threads']} OpenMP "
                      "threads; value = the all-core median"}


def copy_calibration():
    """A plain device-to-device copy of known size (1 GiB read, 1 GiB written
    per copy), run under the FETCH_SIZE / WRITE_SIZE counters to calibrate
    them against known traffic."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copycal", "copies": 3, "bytes_read_per_copy": n * 8,
                      "bytes_written_per_copy": n * 8}), flush=True)


def traffic_record(args):
    """HBM traffic of the bulk stage kernel from four rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE of this bench's throughput mode and of the
    copy calibration), written to profiles/stage_bulk_traffic.json: the
    counters of the last K*3 bulk launches (the stage-timing pass), scaled by
    what the counters read for the 1 GiB copy."""
    import csv
    d = args.pmc_dir
    if not d:
        raise SystemExit("--mode traffic needs --pmc-dir (the folder holding the four counter runs)")

    def col(path, kern):
        with open(path) as f:
            return [float(r["Counter_Value"]) for r in csv.DictReader(f) if kern in r["Kernel_Name"]]

    cf = col(os.path.join(d, "pmc_cfetch", "cfetch_counter_collection.csv"), "copyBuffer")
    cw = col(os.path.join(d, "pmc_cwrite", "cwrite_counter_collection.csv"), "copyBuffer")
    gib_kib = float(1 << 20)
    sf, sw = gib_kib / max(cf), gib_kib / max(cw)
    kern = "k_stage<2, 2, false, "  # the three stage instantiations
    from paper_1905_08717_amd import workloads as W
    n = 3 * W.macro_iters(W.nagumo_2d()) * args.steps  # one bulk launch per stage and iteration
    f = col(os.path.join(d, "pmc_fetch", "fetch_counter_collection.csv"), kern)[-n:]
    w = col(os.path.join(d, "pmc_write", "write_counter_collection.csv"), kern)[-n:]
    fetch = sum(f) / len(f) * sf * 1024
    write = sum(w) / len(w) * sw * 1024

    # the launch configuration of the two counter runs (their bench lines)
    def launch_of(log):
        with open(os.path.join(d, log)) as fh:
            lines = [ln for ln in fh if ln.startswith("{")]
        return json.loads(lines[-1]).get("launch") if lines else None

    launch = launch_of("pmc_fetch.log")
    if launch != launch_of("pmc_write.log"):
        raise SystemExit("the two counter runs used different launch configurations")
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "paper_1905_08717_amd", "csrc", "kernels.hip"), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    rec = {"kernel": kern, "batch": args.batch, "steps": args.steps, "warmup": args.warmup,
           "launches_averaged": len(f), "fetch_scale": round(sf, 4), "write_scale": round(sw, 4),
           "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
           "hbm_bytes_per_launch": round(fetch) + round(write), "kernels_hip_sha256": digest, "launch": launch}
    with open(os.path.join(here, "profiles", "stage_bulk_traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


def paper_tables(args):
    """The paper's own 2D workloads (Sec. 5) on this GPU: inviscid Burgers
    with Dirichlet boundary (t_f 0.9) and Euler Lax-Liu configuration 6
    (t_f 0.25), fixed eps = 0.01, Courant number 0.5, finest levels L; each
    with MRLT/NERK2, MRLT/NERK3 and the uniform scheme (eps = 0: every cell
    is a leaf of level L, identical to FV on the finest grid).  Reports the
    GPU time of each adaptive run as % of the uniform one and the mean
    number of leaves as % of the 4^L finest cells, the paper's "CPU %" and
    "Mem %" columns measured here."""
    import torch
    from paper_1905_08717_amd import mrlt
    from paper_1905_08717_amd import workloads as W

    def run(cfg, q0):
        s = mrlt.Solver(cfg)
        s.load_finest(torch.from_numpy(q0[None]).to("cuda"))
        it = W.macro_iters(cfg)
        mem, steps = 0.0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = 0.0
        while t < cfg["t_final"] * (1 - 1e-12):
            if cfg["pde"] == "burgers":
                dt = W.burgers_dt(cfg)
            else:
                dt = W.euler_dt(cfg, float(s.max_wavespeed()[0]), t)
            s.lt_step(dt)
            t += it * dt
            mem += sum(s.stats()["leaves"])
            steps += 1
        torch.cuda.synchronize()
        return time.perf_counter() - t0, mem / steps / (1 << (2 * cfg["L"])), steps

    rows = []
    for L in [int(x) for x in args.levels.split(",")]:
        for name, mk, q0fn in (("burgers2d", W.burgers_2d, W.burgers_sinsin),
                               ("laxliu6", W.euler_laxliu6, lambda L_: W.euler_quadrants(L_, W.LAXLIU6))):
            q0 = q0fn(L)
            for rk in (2, 3):
                fv_t, _, _ = run(dict(mk(L=L, eps=0.0), rk=rk), q0)
                mr_t, mem, steps = run(dict(mk(L=L), rk=rk), q0)
                rows.append({"problem": name, "L": L, "method": f"MRLT/NERK{rk}", "gpu_s": round(mr_t, 3),
                             "fv_gpu_s": round(fv_t, 3), "time_pct_of_fv": round(100 * mr_t / fv_t, 1),
                             "mem_pct_of_fv": round(100 * mem, 1), "macro_steps": steps})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"mode": "paper", "eps": 0.01, "rows": rows}), flush=True)


def flame_tables(args):
    """The paper's reaction-diffusion problems (Sec. 5) on this GPU: the 1D
    flame (Ze 10, tau 0.8, Courant number 0.5, t_f 5, finest levels from
    --flame-levels) in the frame moving with the front, and the 3D flame ball
    (Le 0.3, kappa 0.1, tau 0.64, Courant number 0.1, t_f 5, L 7 on
    (-15, 15)^3), eps = 0.01.  Methods: MR/RK2 and MR/RK3 (one global step),
    MRLT/NERK2 and MRLT/NERK3, and the uniform scheme of the same RK order
    (eps = 0).  Per method: GPU time as % of the uniform run, mean leaves as
    % of the finest cells, and the discrete L1 error of T, Y and omega
    against the uniform run (x 1e-4, the paper's unit)."""
    import torch
    from paper_1905_08717_amd import mrlt
    from paper_1905_08717_amd import workloads as W

    def omega(cfg, q):
        ze, tau = cfg["ze"], cfg["tau"]
        if cfg["pde"] == "flame":
            u = 1.0 - q[0]
            return 0.5 * ze * ze * u * np.exp(ze * u / (tau * u - 1.0))
        le = cfg["lewis"]
        return ze * ze / (2 * le) * q[1] * np.exp(ze * (q[0] - 1.0) / (1.0 + tau * (q[0] - 1.0)))

    def run(cfg, q0, dt):
        s = mrlt.Solver(cfg)
        s.load_finest(torch.from_numpy(q0[None]).to("cuda"))
        it = W.macro_iters(cfg)
        nmac = int(round(cfg["t_final"] / (it * dt)))
        mem = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(nmac):
            s.lt_step(dt)
            mem += sum(s.stats()["leaves"])
            if (j + 1) % max(1, nmac // 4) == 0:
                print(f"[flames] {cfg['name']} rk={cfg.get('rk', 3)} lt={cfg.get('lt', 1)} eps={cfg['eps']} "
                      f"step {j + 1}/{nmac}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        q = s.reconstruct().cpu().numpy()[0]
        s.close()
        fields = {"T": q[0], "Y": (1.0 - q[0]) if cfg["pde"] == "flame" else q[1], "omega": omega(cfg, q)}
        return el, mem / nmac / (1 << (cfg["dim"] * cfg["L"])), nmac, fields

    cases = [("flame1d", W.flame_1d(L=L), W.flame_front(L)) for L in
             [int(x) for x in args.flame_levels.split(",") if x]]
    if args.flame_ball_level:
        Lb = args.flame_ball_level
        cases.append(("flameball3d", W.flame_ball_3d(L=Lb), W.flame_ball(Lb)))
    rows = []
    for name, base, q0 in cases:
        dt = W.flame_dt(base)
        for rk in (2, 3):
            fv_t, _, _, ref = run(dict(base, rk=rk, eps=0.0), q0, dt)
            for lt in (0, 1):
                el, mem, nmac, f = run(dict(base, rk=rk, lt=lt), q0, dt)
                err = {k: round(1e4 * float(np.abs(f[k] - ref[k]).mean()), 4) for k in f}
                method = f"MRLT/NERK{rk}" if lt else f"MR/RK{rk}"
                rows.append({"problem": name, "L": base["L"], "method": method, "gpu_s": round(el, 3),
                             "fv_gpu_s": round(fv_t, 3), "time_pct_of_fv": round(100 * el / fv_t, 1),
                             "mem_pct_of_fv": round(100 * mem, 2), "l1_err_x1e4_vs_fv": err,
                             "macro_steps": nmac, "dt_L": dt})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"mode": "flames", "eps": 0.01, "rows": rows}), flush=True)


def systems_mode(args):
    """Batched (256 uneven 2D Euler four-quadrant solves) or served (Poisson
    arrivals of Burgers / Nagumo requests) forms; one JSON line."""
    import torch  # noqa: F401
    from paper_1905_08717_amd import systems as S
    if args.mode == "batched":
        reqs = S.batched_euler_requests(args.requests or 256)
        t0 = time.perf_counter()
        b = S.run_batched(reqs)
        solo_reqs = S.batched_euler_requests(args.requests or 256)
        n_solo = min(len(solo_reqs), args.solo_sample)
        a = S.run_one_at_a_time(solo_reqs[:n_solo])
        same = all((r.result is None and q.result is None and r.failed and q.failed) or
                   (r.result is not None and q.result is not None and
                    np.array_equal(r.result[0], q.result[0]) and np.array_equal(r.result[1], q.result[1]))
                   for r, q in zip(reqs[:n_solo], solo_reqs[:n_solo]))
        out = {"metric": "batched solves/s", "value": round(b["solves_per_s"], 3), "unit": "solves/s",
               "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"{len(reqs)} 2D Euler four-quadrant Riemann problems, L in {{7,8,9}}, "
                                      "eps in {1e-2,1e-3,1e-4}, t_final 0.25, per-instance CFL 0.5"},
               "batched": b,
               "one_at_a_time": dict(a, note=f"first {n_solo} of the same requests, each alone"),
               "speedup_vs_one_at_a_time": round(b["solves_per_s"] / a["solves_per_s"], 3),
               "results_identical_to_solo": bool(same), "wall_s": round(time.perf_counter() - t0, 2)}
    else:
        reqs = S.served_requests(args.requests or 200, rate=args.rate,
                                 burgers_levels=tuple(range(10, args.max_burgers_level + 1)))
        r = S.serve(reqs, hbm_budget=args.hbm_budget * 2 ** 30)
        out = {"metric": "served p50/p99 time-to-solution", "value": round(r["p50_s"], 4), "unit": "s",
               "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"{len(reqs)} requests, Poisson {args.rate}/s, half 1D viscous Burgers "
                                      f"(L 10..{args.max_burgers_level}, t_final 0.5), half 2D Nagumo "
                                      "(L 7..9, t_final 0.01), eps log-uniform [1e-4, 1e-2]"},
               "served": r}
    print(json.dumps(out), flush=True)


def euler3d_single(args):
    """The 3D Euler spherical Riemann problem at its stated size (128^3,
    L=7, eps=1e-3, five FP64 fields): one solve, leaf-updates/s over two
    macro steps after one (CFL step from the wave-speed reduction each macro
    step, inside the timed region), then the bulk stage kernel's HBM
    roofline over two macro steps of a fresh load."""
    import torch
    from paper_1905_08717_amd import mrlt
    from paper_1905_08717_amd import workloads as W
    from paper_1905_08717_amd import autotune
    cfg = W.euler_3d(L=7)
    q0 = torch.from_numpy(W.euler_sphere(7)[None]).to("cuda")
    s = mrlt.Solver(cfg)
    stored = None if getattr(args, "no_tune", False) else autotune.lookup(autotune.euler3d_key(7))
    if stored:
        s.set_launch(**stored)

    def run(k, t):
        for _ in range(k):
            dt = W.euler_dt(cfg, s.max_wavespeed()[0], t)
            s.lt_step(dt)
            t += W.macro_iters(cfg) * dt
        return t

    s.load_finest(q0)
    t = run(1, 0.0)
    u0 = total_updates(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(2, t)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    upd = total_updates(s) - u0
    s.load_finest(q0)
    t = run(1, 0.0)
    it0 = s.stage_items()
    s.timing_start("stage_bulk")
    run(2, t)
    ms, launches = s.timing_stop()
    items = s.stage_items() - it0
    m = s.m
    alg = int(items[0]) * 16 * m + int(items[1]) * 24 * m + int(items[2]) * 24 * m
    ach = alg / (ms * 1e-3) / 1e9
    leaves = int(sum(s.stats()["leaves"]))
    items_run = [int(x) for x in s.stage_items()]
    s.close()
    print(f"[bench] 3D Euler L=7: {upd / el:.3e} leaf-updates/s", file=sys.stderr, flush=True)
    # the FP64 roofline of the same launches: FP64 operations per leaf-stage
    # update from the committed instruction-counter run of this mode, when it
    # was taken on the current kernel source
    valu = None
    fp = euler_fp64_record()
    if fp:
        flop = sum(int(items[j]) * fp["flop_per_leaf_stage"][j] for j in range(3))
        tf = flop / (ms * 1e-3) / 1e12
        valu = {"bound": "alu", "achieved": round(tf, 3), "peak": 78.6, "unit": "TFLOP/s",
                "frac": round(tf / 78.6, 5), "flop_per_leaf_stage": fp["flop_per_leaf_stage"],
                "flop_per_byte": round(flop / alg, 2)}
    return {"workload": "euler3d_L7_128^3 spherical Riemann problem, eps=1e-3, one solve, macro steps 2-3 from t=0",
            "leaf_updates_per_s": round(upd / el, 1), "ms_per_macro_step": round(el / 2 * 1e3, 2),
            "leaves": leaves,
            "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(ach / 8000.0, 5), "kernel": "k_stage<3, 3, false, 1|2|3>",
                         "launches": launches, "avg_launch_us": round(ms * 1e3 / max(launches, 1), 3),
                         "alg_bytes_per_leaf_stage": [16 * m, 24 * m, 24 * m]},
            "valu_roofline": valu, "bulk_items_run": items_run,
            "launch": stored, "launch_source": "paper_1905_08717_amd/tuned_launch.json" if stored else "library default"}


def kernels_digest():
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "paper_1905_08717_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def euler_fp64_record():
    """FP64 operations per leaf-stage update of the 3D Euler bulk stage
    kernel (profiles/euler3d_bulk_fp64.json), if taken on the current kernel
    source; otherwise None."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "euler3d_bulk_fp64.json")) as f:
            rec = json.load(f)
        if rec.get("kernels_hip_sha256") != kernels_digest():
            return None
        return rec
    except (OSError, ValueError):
        return None


def fp64_record(args):
    """FP64 operations per leaf-stage update of the 3D Euler bulk stage kernel
    from a rocprofv3 run of `--mode euler3d` with the FP64 instruction counters
    (folder pmc_eul under --pmc-dir, its log pmc_eul.log): (ADD + MUL + TRANS
    + 2 FMA) wave instructions x 64 lanes over all bulk launches of the run,
    divided by the run's leaf-stage updates (an upper bound: lanes outside a
    wave's active mask are counted).  Written to
    profiles/euler3d_bulk_fp64.json."""
    import csv
    d = args.pmc_dir
    if not d:
        raise SystemExit("--mode fp64 needs --pmc-dir")
    tot = [dict(), dict(), dict()]
    with open(os.path.join(d, "pmc_eul", "eul_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = r["Kernel_Name"]
            if not k.startswith("void k_stage<3, 3, false, "):
                continue
            j = int(k.split(",")[3].split(">")[0]) - 1
            tot[j][r["Counter_Name"]] = tot[j].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    with open(os.path.join(d, "pmc_eul.log")) as fh:
        line = [ln for ln in fh if ln.startswith("{")][-1]
    items = json.loads(line)["bulk_items_run"]
    flop = []
    for j in range(3):
        c = tot[j]
        ops = (c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_TRANS_F64"]
               + 2.0 * c["SQ_INSTS_VALU_FMA_F64"]) * 64.0
        flop.append(round(ops / items[j], 1))
    rec = {"kernel": "k_stage<3, 3, false, 1|2|3>", "workload": "bench.py --mode euler3d",
           "counters": [{k: int(v) for k, v in c.items()} for c in tot], "bulk_items_run": items,
           "flop_per_leaf_stage": flop, "kernels_hip_sha256": kernels_digest()}
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "profiles", "euler3d_bulk_fp64.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


def batched_leg(args):
    """The batched configuration: 256 four-quadrant 2D Euler problems (finest
    level from {7, 8, 9}, eps from {1e-2, 1e-3, 1e-4}) to t_final 0.25, all
    in one context of the library's scheduler; against the first 32 of the
    same requests solved one at a time (each alone in a context of its own
    level), whose results must be identical."""
    from paper_1905_08717_amd import systems as S
    reqs = S.batched_euler_requests(256)
    b = S.run_batched(reqs)
    solo = S.batched_euler_requests(256)[:32]
    a = S.run_one_at_a_time(solo)
    same = all((r.failed and q.failed) or
               (r.result is not None and q.result is not None and
                np.array_equal(r.result[0], q.result[0]) and np.array_equal(r.result[1], q.result[1]))
               for r, q in zip(reqs[:32], solo))
    print(f"[bench] batched {b['solves_per_s']:.2f} solves/s, one at a time {a['solves_per_s']:.2f}",
          file=sys.stderr, flush=True)
    return {"workload": "256 2D Euler four-quadrant Riemann problems, L in {7,8,9}, eps in {1e-2,1e-3,1e-4}, "
                        "t_final 0.25, CFL 0.5 per solve",
            "solves_per_s": round(b["solves_per_s"], 3), "seconds": round(b["seconds"], 3),
            "solves": b["solves"], "failed": b["failed"], "macro_steps": b["macro_steps"],
            "hbm_bytes": b["hbm_bytes"],
            "one_at_a_time_solves_per_s": round(a["solves_per_s"], 3),
            "one_at_a_time_sample": "first 32 of the same requests",
            "speedup": round(b["solves_per_s"] / a["solves_per_s"], 3),
            "results_identical_to_one_at_a_time": bool(same)}


def served_leg(args):
    """The served configuration, shortened to 200 requests: Poisson arrivals
    at 200/s, half 1D viscous Burgers (L 10..14, t_final 0.5), half 2D Nagumo
    (L 7..9, t_final 0.01), eps log-uniform in [1e-4, 1e-2]."""
    from paper_1905_08717_amd import systems as S
    reqs = S.served_requests(200, rate=200.0)
    r = S.serve(reqs, hbm_budget=args.hbm_budget * 2 ** 30)
    print(f"[bench] served p50 {r['p50_s']:.2f} s p99 {r['p99_s']:.2f} s", file=sys.stderr, flush=True)
    return dict(r, workload="200 requests (of the configuration's 1000), Poisson 200/s, half 1D viscous Burgers "
                            "L 10..14 t_final 0.5, half 2D Nagumo L 7..9 t_final 0.01, eps log-uniform "
                            "[1e-4, 1e-2]; one class per scheme and finest level, 16 slots each")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=4.0)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 3D Euler, batched and served legs of the default line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["throughput", "batched", "served", "copycal", "traffic", "paper",
                                       "flames", "cpu-oracle", "euler3d", "fp64"],
                    default="throughput")
    ap.add_argument("--levels", default="8,9,10", help="paper mode: finest levels")
    ap.add_argument("--flame-levels", default="11,12", help="flames mode: finest levels of the 1D flame")
    ap.add_argument("--flame-ball-level", type=int, default=7, help="flames mode: 3D flame ball L (0: skip)")
    ap.add_argument("--pmc-dir", default="", help="traffic mode: folder of the four counter runs (required)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-solve reference run")
    ap.add_argument("--tune", action="store_true", help="search the launch configuration before timing")
    ap.add_argument("--no-tune", action="store_true", help="library default launch configuration")
    ap.add_argument("--launch", default="", help="list,iface,comp grid caps")
    ap.add_argument("--requests", type=int, default=0)
    ap.add_argument("--solo-sample", type=int, default=32)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--max-burgers-level", type=int, default=14)
    ap.add_argument("--hbm-budget", type=float, default=64.0, help="GiB for resident solves")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (--gpus 1); independent solves would shard "
              "across GPUs by instance, which is not built here", file=sys.stderr)
        sys.exit(2)

    if args.mode == "cpu-oracle":
        cpu_oracle_leg(args.cpu_seconds)
        return
    if args.mode == "fp64":
        fp64_record(args)
        return
    if args.mode == "euler3d":
        print(json.dumps(euler3d_single(args)), flush=True)
        return
    if args.mode == "copycal":
        copy_calibration()
        return
    if args.mode == "traffic":
        traffic_record(args)
        return
    if args.mode == "paper":
        paper_tables(args)
        return
    if args.mode == "flames":
        flame_tables(args)
        return
    if args.mode != "throughput":
        systems_mode(args)
        return

    import torch
    from paper_1905_08717_amd import mrlt
    from paper_1905_08717_amd import workloads as W

    cfg = W.nagumo_2d()
    B = args.batch
    dt = W.nagumo_dt(cfg)
    q0 = np.stack([W.nagumo_front(cfg["L"], W.SEED + i) for i in range(B)])
    q0d = torch.from_numpy(q0).to("cuda")
    s = mrlt.Solver(cfg, n_inst=B)
    # launch configuration (results do not depend on it): given, searched
    # now (untimed), the stored measured setting of this workload, or the
    # library default
    from paper_1905_08717_amd import autotune
    tuned, source = None, "library default"
    stored = autotune.lookup(autotune.nagumo_key(cfg["L"], B))
    if args.launch:
        lg, ig, cg = (int(v) for v in args.launch.split(","))
        s.set_launch(list_grid=lg, iface_grid=ig, comp_grid=cg)
        source = "--launch"
    elif args.tune:
        r = autotune.tune(s, q0d, dt, passes=1)
        tuned = {"launch": r["best"], "ms_per_step_default": round(1e3 * r["default"], 2),
                 "ms_per_step_tuned": round(1e3 * r["seconds_per_step"], 2), "trials": len(r["trials"])}
        source = "tuned in this run"
        print(f"[bench] launch {tuned}", file=sys.stderr, flush=True)
    elif stored and not args.no_tune:
        s.set_launch(**stored)
        source = "paper_1905_08717_amd/tuned_launch.json"
    s.load_finest(q0d)
    for _ in range(args.warmup):
        s.lt_step(dt)

    # timed region: K macro steps over the batch
    u0 = total_updates(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.lt_step(dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    upd = total_updates(s) - u0
    value = upd / el
    leaves = leaf_counts(s)

    # roofline of the dominant kernel, the bulk RK stage kernel: HIP events
    # around each of its launches over the same number of macro steps, and
    # its leaf-stage updates counted on the device; algorithmic bytes per
    # leaf-stage update 16m (stage 1), 24m (stages 2, 3)
    it0 = s.stage_items()
    s.timing_start("stage_bulk")
    for _ in range(args.steps):
        s.lt_step(dt)
    ms, launches = s.timing_stop()
    items = s.stage_items() - it0
    m = s.m
    alg_bytes = int(items[0]) * 16 * m + int(items[1]) * 24 * m + int(items[2]) * 24 * m
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 5), "traffic": stage_traffic(B, s.get_launch()["list_grid"]),
                "kernel": "k_stage<2, 2, false, 1|2|3> (bulk RK stage kernel, all levels of a stage)",
                "launches": launches, "avg_launch_us": round(ms * 1e3 / max(launches, 1), 3),
                "alg_bytes_per_launch": round(alg_bytes / max(launches, 1), 1),
                "leaf_stage_updates": [int(x) for x in items],
                "alg_bytes_per_leaf_stage": [16 * m, 24 * m, 24 * m]}

    # single-solve reference (one instance), same work per macro step
    single, stored1 = None, None
    if not args.no_single:
        s1 = mrlt.Solver(cfg, n_inst=1)
        stored1 = autotune.lookup(autotune.nagumo_key(cfg["L"], 1))
        if stored1 and not args.no_tune:
            s1.set_launch(**stored1)
        s1.load_finest(torch.from_numpy(q0[:1]).to("cuda"))
        s1.lt_step(dt)
        a = total_updates(s1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            s1.lt_step(dt)
        torch.cuda.synchronize()
        single = round((total_updates(s1) - a) / (time.perf_counter() - t1), 1)

    out = {
        "metric": "leaf cell-updates/s", "value": round(value, 1), "unit": "leaf-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"nagumo2d_L9_512x512_eps1e-3 batch of {B} seeded fronts "
                               f"(one macro step = 128 fine iterations per instance)",
                   "dim": 2, "L": 9, "l0": 2, "eps": 1e-3, "batch": B, "dt_L": dt,
                   "leaves_per_level_total": [int(x) for x in leaves[:10]]},
        "roofline": roofline,
        # the whole macro step against the same floor: 64m algorithmic bytes
        # per leaf-update (16m + 24m + 24m over the three stages)
        "whole_step": {"bound": "hbm", "achieved": round(upd * 64 * s.m / el / 1e9, 2), "peak": 8000.0,
                       "unit": "GB/s", "frac": round(upd * 64 * s.m / el / 1e9 / 8000.0, 5),
                       "alg_bytes_per_leaf_update": 64 * s.m},
        "launch": s.get_launch(),
        "launch_source": source,
        "autotune": tuned,
        "single_solve_leaf_updates_per_s": single,
        "single_solve_launch": (stored1 if (single is not None and stored1 and not args.no_tune) else None),
        "solves_macro_steps_per_s": round(B * args.steps / el, 2),
    }
    del s
    torch.cuda.empty_cache()
    if not args.no_configs:
        out["euler3d"] = euler3d_single(args)
        out["batched"] = batched_leg(args)
        out["served"] = served_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
