"""Pins of the MR scheme with a global time step (lt = 0), the paper's
comparison method MR/RK (Sec. 1, Sec. 5): every leaf advances by the same dt,
virtual cells and the finer side of refined faces are taken at the same
stage time (projections of the children's stage values), so the scheme keeps
the order of the RK method (Table 1: MR/RK3 3.00, MR/RK2 2.00)."""
import json
import math
import os

import numpy as np
import pytest

from paper_1905_08717_amd import workloads as W
from tests import fv_uniform as FV
from tests.test_oracle_pins import GOLDEN, _gauss_avg, tree_1d, tree_2d
from tests.trees import box_average_poly, build_tree, leaf_arrays, leaf_key


def test_single_level_tree_steps_with_global_dt(oracle_mod):
    L, lev, l0 = 7, 5, 2
    cfg = dict(W.burgers_1d(L=L, eps=0.0), lt=0, remesh=0)
    o = oracle_mod.Oracle(cfg)
    q0 = W.burgers_sine(lev) + 0.3
    leaves = build_tree(1, lev, l0, lambda c: lev)
    keys = np.array([leaf_key(lev, 1, x) for _, x in leaves], dtype=np.uint64)
    o.set_leaves(keys, np.array([[q0[0, x[0]] for _, x in leaves]]))
    dt = 1e-3
    o.lt_step(dt)
    q = q0.copy()
    for _ in range(W.macro_iters(cfg)):
        q = FV.rk3_step(cfg, q, lev, dt)
    _, got = o.get_leaves()
    assert np.array_equal(got, q)


@pytest.mark.parametrize("rk", [2, 3])
@pytest.mark.parametrize("dim", [1, 2])
def test_global_step_exact_for_linear_in_time_quadratic_diffusion(oracle_mod, rk, dim):
    L, l0 = (8, 6) if dim == 1 else (7, 5)
    dt = 0.2 / (1 << L) ** 2
    cfg = dict(dim=dim, L=L, l0=l0, eps=0.0, pde="linear", nu=1.0, k_react=0.0, bc="neumann",
               remesh=0, rk=rk, lt=0)
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


def test_global_step_mass_conserved(oracle_mod):
    cfg = dict(W.burgers_1d(L=9, eps=1e-3), lt=0)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.burgers_sine(9) + 0.5)
    m0 = o.stats()["mass"][0]
    for _ in range(3):
        o.lt_step(0.5 * (1.0 / 512) / 1.6)
    assert abs(o.stats()["mass"][0] - m0) < 1e-13


def _run(oracle_mod, dt, rk):
    cfg = dict(dim=1, L=9, l0=8, eps=0.0, pde="advection", adv_vel=[1.0, 0, 0], bc="periodic",
               recon=2, reflux=0, remesh=0, rk=rk, lt=0)
    o = oracle_mod.Oracle(cfg)
    a9, a8 = _gauss_avg(9), _gauss_avg(8)
    leaves = [(9, (i,)) for i in range(256)] + [(8, (i,)) for i in range(128, 256)]
    leaves.sort(key=lambda lx: leaf_key(lx[0], 1, lx[1]))
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [(a9 if lev == 9 else a8)[x[0]]])
    o.set_leaves(keys, vals)
    for _ in range(int(round(1.0 / dt)) // 2):
        o.lt_step(dt)
    return o.reconstruct()[0]


@pytest.mark.parametrize("rk,key", [(3, "MR/RK3"), (2, "MR/RK2")])
def test_table1_mr_orders(oracle_mod, rk, key):
    gold = json.load(open(os.path.join(GOLDEN, "table1_orders.json")))
    q = [_run(oracle_mod, 1.6e-4 / 2 ** j, rk) for j in range(3)]
    p = math.log2(np.abs(q[0] - q[1]).sum() / np.abs(q[1] - q[2]).sum())
    assert abs(p - gold[key][0]) < 0.05, p
