"""Pins of the MRLT/NERK2 variant (rk = 2): compact RK2 with the NERK
theta = 1/2 value (Sec. 3), synchronisation of Sec. 4 with q_{1/2} in place
of q** (Sec. 4.3), Table 1 orders FV/RK2 and MRLT/NERK2 (Sec. 4.5)."""
import json
import math
import os

import numpy as np
import pytest

from paper_1905_08717_amd import workloads as W
from tests import fv_uniform as FV
from tests.test_oracle_pins import GOLDEN, _gauss_avg, tree_1d, tree_2d
from tests.trees import box_average_poly, leaf_arrays, leaf_key


@pytest.mark.parametrize("name,cfg,q0fn,dt", [
    ("burgers1d", W.burgers_1d(L=7, eps=0.0), lambda: W.burgers_sine(7) + 0.25, 1e-3),
    ("nagumo2d", W.nagumo_2d(L=5, eps=0.0), lambda: W.nagumo_front(5), 1e-5),
    ("euler2d", W.euler_2d(L=5, eps=0.0), lambda: W.euler_quadrants_seeded(5, W.SEED), 1e-3),
])
def test_eps0_equals_uniform_fv_rk2(oracle_mod, name, cfg, q0fn, dt):
    cfg = dict(cfg, rk=2)
    o = oracle_mod.Oracle(cfg)
    q0 = q0fn()
    o.load_finest(q0)
    o.lt_step(dt)
    q = FV.to_grid(cfg, q0.copy(), cfg["L"])
    for _ in range(W.macro_iters(cfg)):
        q = FV.rk2_step(cfg, q, cfg["L"], dt)
    assert np.array_equal(o.reconstruct(), q.reshape(o.reconstruct().shape))


def test_rk2_amplification_polynomial_per_level(oracle_mod):
    L, l0, k, dt = 8, 6, -3.0, 0.01
    cfg = dict(dim=1, L=L, l0=l0, eps=0.0, pde="linear", nu=0.0, k_react=k, bc="periodic", remesh=0, rk=2)
    leaves = tree_1d(L, l0)
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [1.0])
    o = oracle_mod.Oracle(cfg)
    o.set_leaves(keys, vals)
    o.lt_step(dt)
    _, got = o.get_leaves()
    for j, (lev, x) in enumerate(leaves):
        z = k * dt * 2 ** (L - lev)
        assert got[0, j] == pytest.approx((1 + z + z * z / 2) ** (2 ** (lev - l0)), rel=2e-15)


@pytest.mark.parametrize("dim", [1, 2])
def test_rk2_sync_exact_for_linear_in_time_quadratic_diffusion(oracle_mod, dim):
    L, l0 = (8, 6) if dim == 1 else (7, 5)
    dx = 1.0 / (1 << L)
    dt = 0.2 * dx * dx
    cfg = dict(dim=dim, L=L, l0=l0, eps=0.0, pde="linear", nu=1.0, k_react=0.0, bc="neumann",
               remesh=0, rk=2)
    leaves = tree_1d(L, l0) if dim == 1 else tree_2d(L, l0)
    keys, vals = leaf_arrays(dim, leaves, lambda lev, x: [box_average_poly(dim, lev, x, [1.0] * dim)])
    o = oracle_mod.Oracle(cfg)
    o.set_leaves(keys, vals)
    for _ in range(2):
        o.lt_step(dt)
    t = 2 * W.macro_iters(cfg) * dt
    _, got = o.get_leaves()
    n = 0
    for j, (lev, x) in enumerate(leaves):
        if max((x[a] + 1) / (1 << lev) for a in range(dim)) > 0.75:
            continue
        assert got[0, j] == pytest.approx(box_average_poly(dim, lev, x, [1.0] * dim) + 2 * dim * t, abs=2e-13)
        n += 1
    assert n > 20


def test_rk2_mass_conserved(oracle_mod):
    cfg = dict(W.burgers_1d(L=9, eps=1e-3), rk=2)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.burgers_sine(9) + 0.5)
    m0 = o.stats()["mass"][0]
    for _ in range(5):
        o.lt_step(0.5 * (1.0 / 512) / 1.6)
    assert abs(o.stats()["mass"][0] - m0) < 1e-13


def _run(oracle_mod, dt, uniform):
    cfg = dict(dim=1, L=9, l0=8, eps=0.0, pde="advection", adv_vel=[1.0, 0, 0], bc="periodic",
               recon=2, reflux=0, remesh=0, rk=2)
    o = oracle_mod.Oracle(cfg)
    a9, a8 = _gauss_avg(9), _gauss_avg(8)
    leaves = [(9, (i,)) for i in range(512)] if uniform else \
        [(9, (i,)) for i in range(256)] + [(8, (i,)) for i in range(128, 256)]
    leaves.sort(key=lambda lx: leaf_key(lx[0], 1, lx[1]))
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [(a9 if lev == 9 else a8)[x[0]]])
    o.set_leaves(keys, vals)
    for _ in range(int(round(1.0 / dt)) // 2):
        o.lt_step(dt)
    return o.reconstruct()[0]


def _order(oracle_mod, dt, uniform):
    q = [_run(oracle_mod, dt / 2 ** j, uniform) for j in range(3)]
    return math.log2(np.abs(q[0] - q[1]).sum() / np.abs(q[1] - q[2]).sum())


def test_table1_rk2_orders(oracle_mod):
    gold = json.load(open(os.path.join(GOLDEN, "table1_orders.json")))
    assert abs(_order(oracle_mod, 1.6e-4, True) - gold["FV/RK2"][0]) < 0.05
    assert abs(_order(oracle_mod, 1.6e-4, False) - gold["MRLT/NERK2"][0]) < 0.1
