"""The systems forms through the C ABI (mr_batch_*, mr_load_inst, the
allocator callbacks): every call exercised, results of batched and served
solves equal to the same solves alone bit for bit, and sampled solves equal
to the CPU oracle run to their final time with the same step rule."""
import math

import numpy as np
import pytest

from paper_1905_08717_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="module")
def mods():
    if not _gpu_ok():
        pytest.skip("no GPU")
    from oracle import mro
    from paper_1905_08717_amd import mrlt
    mrlt.load_library()
    return mro, mrlt


def oracle_solve(mro, cfg, q0, t_final, cfl=0.5):
    """The oracle run with the batch's step rule: per macro step
    dt = min(cfl / (w/dx + 2 d nu/dx^2 + 0.8 k [Nagumo]), (t_final - t) / N),
    evaluated in the same order."""
    o = mro.Oracle(cfg)
    o.load_finest(q0)
    L, l0, dim = cfg["L"], cfg.get("l0", 2), cfg["dim"]
    dx = (cfg.get("hi", [1.0] * 3)[0] - cfg.get("lo", [0.0] * 3)[0]) / math.ldexp(1.0, L)
    n_it = math.ldexp(1.0, L - l0)
    nu = cfg.get("nu", 0.0) if cfg["pde"] in ("burgers", "nagumo", "linear") else 0.0
    t = 0.0
    steps = 0
    while t < t_final * (1.0 - 1e-12):
        rate = o.max_wavespeed() / dx + 2.0 * dim * nu / (dx * dx)
        if cfg["pde"] == "nagumo":
            rate += 0.8 * cfg["k_react"]
        dt = cfl / rate if rate > 0.0 else (t_final - t) / n_it
        dt = min(dt, (t_final - t) / n_it)
        o.lt_step(dt)
        t = t + n_it * dt
        steps += 1
    return o, steps


def test_batch_calls_and_results_against_the_oracle(mods):
    mro, mrlt = mods
    rd = W.nagumo_2d(L=7, eps=1e-3)
    bu = W.burgers_1d(L=9, eps=1e-3)
    b = mrlt.Batch([(rd, 7, 2), (bu, 9, 1)], hbm_budget=8 * 2 ** 30)
    jobs = [(rd, 6, 1e-3, W.nagumo_front(6, W.SEED + 1), 1e-3),
            (rd, 7, 3e-3, W.nagumo_front(7, W.SEED + 2), 1e-3),
            (bu, 9, 1e-3, W.burgers_sine(9, 0.1), 0.05)]
    slots = [b.admit(dict(c, L=L, eps=e), L, e, tf, q) for c, L, e, q, tf in jobs]
    assert slots == [0, 1, 2]
    assert b.admit(dict(bu, L=9), 9, 1e-3, 0.05, W.burgers_sine(9)) is None     # class full
    with pytest.raises(mrlt.MrError) as e:
        b.admit(W.euler_2d(L=6), 6, 1e-3, 0.1, W.euler_quadrants_seeded(6, 1))  # no such class
    assert e.value.code == mrlt.EINVAL
    assert all(b.slot_info(s)["state"] == mrlt.SLOT_RUNNING for s in slots)
    assert b.footprint() > 0
    print("[systems] batch of 3 solves in 2 classes", flush=True)
    done = []
    while len(done) < 3:
        b.step()
        done += b.poll()
    assert sorted(done) == slots
    for (c, L, e, q, tf), s in zip(jobs, slots):
        info = b.slot_info(s)
        assert info["state"] == mrlt.SLOT_DONE and abs(info["t"] - tf) <= 1e-12 * tf
        kg, vg = b.get_leaves(s, 1)
        o, steps = oracle_solve(mro, dict(c, L=L, eps=e), q, tf)
        ko, vo = o.get_leaves()
        assert steps == info["macro_steps"]
        assert np.array_equal(kg, ko) and np.array_equal(vg, vo), (s, L)
        b.release(s)
        assert b.slot_info(s)["state"] == mrlt.SLOT_FREE
    assert b.admit(dict(bu, L=8), 8, 1e-3, 0.02, W.burgers_sine(8)) == 2          # released slot reused
    b.close()


def test_uneven_batch_equals_one_at_a_time_and_oracle(mods):
    # the batched configuration's shape: four-quadrant 2D Euler problems of
    # finest level 7, 8 and 9 in one class; results bit for bit equal to
    # each solve alone in a context of its own level, and to the oracle
    mro, mrlt = mods
    import copy
    from paper_1905_08717_amd import systems as S
    pool = S.batched_euler_requests(30)
    reqs = [r for L in (7, 8, 9) for r in [q for q in pool if q.cfg["L"] == L][:3]]
    for r in reqs:
        r.t_final = 0.05
    alone = copy.deepcopy(reqs)
    out = S.run_batched(reqs)
    S.run_one_at_a_time(alone)
    assert out["solves"] + out["failed"] == len(reqs)
    for a, b in zip(reqs, alone):
        assert a.failed == b.failed
        if not a.failed:
            assert np.array_equal(a.result[0], b.result[0]) and np.array_equal(a.result[1], b.result[1])
    sample = {}
    for r in reqs:
        if not r.failed:
            sample.setdefault(r.cfg["L"], r)
    assert len(sample) == 3
    for L, r in sorted(sample.items()):
        print(f"[systems] oracle to t_final, L={L}", flush=True)
        o, steps = oracle_solve(mro, r.cfg, r.q0, r.t_final)
        ko, vo = o.get_leaves()
        assert steps == r.macro_steps
        assert np.array_equal(r.result[0], ko) and np.array_equal(r.result[1], vo), L


def test_served_results_equal_solo(mods):
    # continuous batching: every served result equals the same request alone
    _, mrlt = mods
    import copy
    from paper_1905_08717_amd import systems as S
    served = S.served_requests(16, rate=400.0, burgers_levels=(9, 10), rd_levels=(6, 7))
    for r in served:
        r.t_final = r.t_final / 20
    alone = copy.deepcopy(served)
    out = S.serve(served, hbm_budget=8 * 2 ** 30, slots=4)
    assert out["requests"] == 16 and out["failed"] == 0 and out["p99_s"] >= out["p50_s"] > 0
    S.run_one_at_a_time(alone)
    for a, b in zip(served, alone):
        assert a.result is not None and b.result is not None
        assert np.array_equal(a.result[0], b.result[0]) and np.array_equal(a.result[1], b.result[1]), a.rid


def test_admission_by_device_footprint(mods):
    # a budget that holds one class context at a time: the second class waits
    # while the first runs, and gets the memory once the first is idle
    _, mrlt = mods
    bu = W.burgers_1d(L=12, eps=1e-3)
    rd = W.nagumo_2d(L=8, eps=1e-3)
    probe = mrlt.Batch([(bu, 12, 2), (rd, 8, 2)], hbm_budget=64 * 2 ** 30)
    probe.admit(bu, 12, 1e-3, 1e-3, W.burgers_sine(12))
    fa = probe.footprint()
    probe.admit(rd, 8, 1e-3, 1e-5, W.nagumo_front(8))
    fb = probe.footprint() - fa
    probe.close()
    assert fa > 0 and fb > 0
    b = mrlt.Batch([(bu, 12, 2), (rd, 8, 2)], hbm_budget=max(fa, fb) + (1 << 20))
    sa = b.admit(bu, 12, 1e-3, 2e-3, W.burgers_sine(12))
    assert sa is not None and b.footprint() == fa
    assert b.admit(rd, 8, 1e-3, 1e-5, W.nagumo_front(8)) is None      # does not fit beside it
    while b.slot_info(sa)["state"] == mrlt.SLOT_RUNNING:
        b.step()
    assert b.poll() == [sa]
    keys, vals = b.get_leaves(sa, 1)                                      # kept on the host
    sb = b.admit(rd, 8, 1e-3, 1e-5, W.nagumo_front(8))                  # the idle context made room
    assert sb is not None and b.footprint() == fb
    k2, v2 = b.get_leaves(sa, 1)
    assert np.array_equal(keys, k2) and np.array_equal(vals, v2)
    b.close()


def test_contexts_on_the_torch_caching_allocator(mods):
    _, mrlt = mods
    import torch
    cfg = W.nagumo_2d(L=7)
    q = W.nagumo_front(7)
    dt = W.nagumo_dt(cfg)
    plain = mrlt.Solver(cfg)
    before = torch.cuda.memory_allocated()
    pooled = mrlt.Solver(cfg, alloc=mrlt.torch_allocator())
    grown = torch.cuda.memory_allocated() - before
    assert grown >= pooled.footprint() > 0
    assert plain.footprint() == pooled.footprint()
    for s in (plain, pooled):
        s.load_finest(q[None])
        s.lt_step(dt)
        s.lt_step(dt)
    ka, va = plain.get_leaves()
    kb, vb = pooled.get_leaves()
    assert np.array_equal(ka, kb) and np.array_equal(va, vb)
    m1 = torch.cuda.memory_allocated()
    pooled.close()
    assert m1 - torch.cuda.memory_allocated() == grown      # every block went back to torch
    plain.close()


def test_batched_configuration_samples_to_t_final(mods):
    # the batched configuration (2D Euler four-quadrant problems, finest level
    # drawn from {7, 8, 9}, eps from {1e-2, 1e-3, 1e-4}, t_final 0.25): one
    # request of each level run batched with three more, to t_final, against
    # the oracle with the same step rule
    mro, mrlt = mods
    from paper_1905_08717_amd import systems as S
    pool = S.batched_euler_requests(30)
    sample = [[q for q in pool if q.cfg["L"] == L][0] for L in (7, 8, 9)]
    others = [q for q in pool if q not in sample][:3]
    out = S.run_batched(sample + others)
    assert out["failed"] == 0
    for r in sample:
        print(f"[systems] request {r.rid} (L={r.cfg['L']}, eps={r.eps}) against the oracle to t=0.25", flush=True)
        o, steps = oracle_solve(mro, r.cfg, r.q0, r.t_final)
        ko, vo = o.get_leaves()
        assert steps == r.macro_steps
        assert np.array_equal(r.result[0], ko) and np.array_equal(r.result[1], vo), r.rid
