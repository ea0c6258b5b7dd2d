"""Pins of the oracle's macro step against what the paper and the mathematics fix.

* eps = 0 keeps the full tree, so one macro step must be the uniform
  finite-volume / compact RK3 scheme on the finest level (bit for bit, same
  expression trees) -- MR analysis of Sec. 2 with nothing thresholded.
* A frozen single-level tree at level l must be FV/RK3 at level l with the
  local step 2^{L-l} dt (eq. dt).
* The compact RK3 forms (Sec. 3) have the amplification polynomial
  1 + z + z^2/2 + z^3/6 (Sec. 4.4).
* Every synchronisation value of Sec. 4 (first-order theta=1/2 values,
  eqs. projleaf/projnode, refreshRk2, ProjRK3equations1/2, rk3proj and the
  end value of Sec. 4.3) is exact for solutions linear in time, and the
  prediction is exact for quadratics in space: u = x^2 (+ y^2) under
  u_t = nu Lap u evolves as u + 2 d nu t exactly on any graded tree.
* Constant states are preserved (all sync coefficients sum to one).
* Mass is conserved to round-off with the conservative flux accumulation.
* Table 1 of Sec. 4.5: FV/RK3 order 3, MRLT/NERK3 order 2.
* Homogeneous Dirichlet (the paper's 2D Burgers problem): eps = 0 is the
  uniform scheme with odd-mirrored boundary cells, and the heat equation
  converges at second order to exp(-pi^2 t) sin(pi x).
* Viscous Burgers converges to the Cole-Hopf solution; the 1D Euler shock
  tube converges to the exact Riemann solution; a planar 3D problem reduces
  to 1D exactly; the spherical 3D problem keeps octahedral symmetry.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1905_08717_amd import workloads as W
from tests import exact_solutions as X
from tests import fv_uniform as FV
from tests.trees import box_average_poly, build_tree, leaf_arrays, leaf_key

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# eps = 0 and single-level trees reduce to uniform FV/RK3

CASES_T5 = [
    ("burgers1d", W.burgers_1d(L=7, eps=0.0), lambda c: W.burgers_sine(7) + 0.25, 2e-3, 2),
    ("nagumo2d", W.nagumo_2d(L=5, eps=0.0), lambda c: W.nagumo_front(5), 2e-5, 1),
    ("euler2d", W.euler_2d(L=5, eps=0.0), lambda c: W.euler_quadrants_seeded(5, W.SEED), 1e-3, 1),
    ("euler3d", W.euler_3d(L=4, eps=0.0), lambda c: W.euler_sphere(4), 5e-3, 1),
    ("euler1d", W.euler_1d(L=6, eps=0.0), lambda c: W.euler_shock_tube(6), 1e-3, 2),
    ("burgers2d_dirichlet", W.burgers_2d(L=5, eps=0.0), lambda c: W.burgers_sinsin(5), 4e-3, 1),
    ("heat1d_dirichlet", W.linear_1d_dirichlet(L=6), lambda c: W.sine_half(6) + 0.0, 2e-5, 2),
]


@pytest.mark.parametrize("name,cfg,q0fn,dt,nmac", CASES_T5, ids=[c[0] for c in CASES_T5])
def test_eps0_equals_uniform_fv_rk3(oracle_mod, name, cfg, q0fn, dt, nmac):
    o = oracle_mod.Oracle(cfg)
    q0 = q0fn(cfg)
    o.load_finest(q0)
    for _ in range(nmac):
        o.lt_step(dt)
    got = o.reconstruct()
    q = FV.to_grid(cfg, q0.copy(), cfg["L"])
    for _ in range(nmac * W.macro_iters(cfg)):
        q = FV.rk3_step(cfg, q, cfg["L"], dt)
    assert np.array_equal(got, q.reshape(got.shape))
    st = o.stats()
    assert st["leaf_updates"] == nmac * W.macro_iters(cfg) * q0.shape[1]


@pytest.mark.parametrize("dim,lev", [(1, 5), (2, 4)])
def test_single_level_tree_equals_fv_at_that_level(oracle_mod, dim, lev):
    L, l0 = lev + 2, 2
    cfg = (W.burgers_1d(L=L, eps=0.0) if dim == 1 else W.nagumo_2d(L=L, eps=0.0))
    cfg["remesh"] = 0
    o = oracle_mod.Oracle(cfg)
    q0 = (W.burgers_sine(lev) + 0.3) if dim == 1 else W.nagumo_front(lev)
    leaves = build_tree(dim, lev, l0, lambda c: lev)
    keys = np.array([leaf_key(lev, dim, x) for _, x in leaves], dtype=np.uint64)
    n = 1 << lev
    vals = np.array([[q0[0, sum(x[a] * n ** a for a in range(dim))] for _, x in leaves]])
    o.set_leaves(keys, vals)
    dt = 1e-3 if dim == 1 else 1e-6
    o.lt_step(dt)
    got_keys, got = o.get_leaves()
    assert np.array_equal(got_keys, keys)
    q = FV.to_grid(cfg, q0.copy(), lev)
    h = dt * 2 ** (L - lev)
    for _ in range(2 ** (lev - l0)):
        q = FV.rk3_step(cfg, q, lev, h)
    qf = q.reshape(1, -1)
    ref = np.array([[qf[0, sum(x[a] * n ** a for a in range(dim))] for _, x in leaves]])
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------------------
# designed multi-level trees (frozen) for the synchronisation pins


def tree_1d(L=8, l0=6):
    def levfn(c):
        x = c[0]
        if 0.375 <= x < 0.5:
            return 8
        if 0.25 <= x < 0.625:
            return 7
        return 6
    return build_tree(1, L, l0, levfn)


def tree_2d(L=7, l0=5):
    def levfn(c):
        x, y = c
        if 0.375 <= x < 0.625 and 0.375 <= y < 0.625:
            return 7
        if 0.25 <= x < 0.75 and 0.25 <= y < 0.75:
            return 6
        return 5
    return build_tree(2, L, l0, levfn)


def g_rk3(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0


def test_rk3_amplification_polynomial_per_level(oracle_mod):
    # dq/dt = k q per cell (no flux): each leaf must advance by
    # g(k h_l)^(2^{l-l0}) in one macro step, h_l = 2^{L-l} dt (eq. dt).
    L, l0, k, dt = 8, 6, -3.0, 0.01
    cfg = dict(dim=1, L=L, l0=l0, eps=0.0, pde="linear", nu=0.0, k_react=k,
               bc="periodic", remesh=0)
    leaves = tree_1d(L, l0)
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [1.0])
    o = oracle_mod.Oracle(cfg)
    o.set_leaves(keys, vals)
    o.lt_step(dt)
    _, got = o.get_leaves()
    for j, (lev, x) in enumerate(leaves):
        z = k * dt * 2 ** (L - lev)
        assert got[0, j] == pytest.approx(g_rk3(z) ** (2 ** (lev - l0)), rel=2e-15)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("reflux", [0, 1])
def test_sync_exact_for_linear_in_time_quadratic_diffusion(oracle_mod, dim, reflux):
    # u = |x|^2 solves u_t = nu Lap u with u_t = 2 d nu constant.  The
    # prediction is exact for quadratics and all time interpolations and
    # extrapolations of Sec. 4 are exact for linear-in-time data, so the
    # multilevel LT macro step must reproduce u + 2 d nu t exactly (to
    # rounding) away from the x=1 / y=1 boundaries (x=0 and y=0 are exact
    # because |x|^2 is even there).  Any wrong time level, dropped term or
    # wrong coefficient in a synchronisation formula breaks it.
    L, l0 = (8, 6) if dim == 1 else (7, 5)
    nu = 1.0
    dx = 1.0 / (1 << L)
    dt = 0.2 * dx * dx / nu
    cfg = dict(dim=dim, L=L, l0=l0, eps=0.0, pde="linear", nu=nu, k_react=0.0,
               bc="neumann", remesh=0, reflux=reflux)
    leaves = tree_1d(L, l0) if dim == 1 else tree_2d(L, l0)
    levels = sorted({lev for lev, _ in leaves})
    assert len(levels) == 3
    keys, vals = leaf_arrays(dim, leaves, lambda lev, x: [box_average_poly(dim, lev, x, [1.0] * dim)])
    o = oracle_mod.Oracle(cfg)
    o.set_leaves(keys, vals)
    nmac = 2
    for _ in range(nmac):
        o.lt_step(dt)
    t = nmac * W.macro_iters(cfg) * dt
    _, got = o.get_leaves()
    checked = 0
    for j, (lev, x) in enumerate(leaves):
        hi = [(x[a] + 1) / (1 << lev) for a in range(dim)]
        if max(hi) > 0.75:
            continue
        exact = box_average_poly(dim, lev, x, [1.0] * dim) + 2 * dim * nu * t
        assert got[0, j] == pytest.approx(exact, abs=2e-13), (lev, x)
        checked += 1
    assert checked > 20


@pytest.mark.parametrize("pde", ["burgers", "euler2d"])
def test_constant_state_preserved_on_multilevel_tree(oracle_mod, pde):
    if pde == "burgers":
        cfg = dict(dim=1, L=8, l0=6, eps=0.0, pde="burgers", nu=1e-3, bc="periodic", remesh=0)
        leaves = tree_1d()
        state = [0.75]
    else:
        cfg = dict(dim=2, L=7, l0=5, eps=0.0, pde="euler", gamma=1.4, bc="periodic", remesh=0)
        leaves = tree_2d()
        state = W.euler_state(1.0, 0.5, -0.25, 0.0, 1.0, 1.4, dim=2)
    keys, vals = leaf_arrays(cfg["dim"], leaves, lambda lev, x: state, m=len(state))
    o = oracle_mod.Oracle(cfg)
    o.set_leaves(keys, vals)
    for _ in range(2):
        o.lt_step(1e-3)
    _, got = o.get_leaves()
    for k in range(len(state)):
        assert np.allclose(got[k], state[k], rtol=4e-16, atol=4e-16)


# ---------------------------------------------------------------------------
# conservation (conservative flux accumulation at level interfaces)


def _mass(o):
    return np.array(o.stats()["mass"])


def test_mass_conserved_adaptive_burgers(oracle_mod):
    cfg = W.burgers_1d(L=9, eps=1e-3)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.burgers_sine(9) + 0.5)
    m0 = _mass(o)
    dt = 0.5 * (1.0 / 512) / 1.6
    levels_seen = set()
    for _ in range(6):
        o.lt_step(dt)
        levels_seen |= {i for i, v in enumerate(o.stats()["leaves"]) if v}
    assert len(levels_seen) >= 3
    assert abs(_mass(o)[0] - m0[0]) < 1e-13


def test_mass_drifts_without_reflux(oracle_mod):
    cfg = W.burgers_1d(L=9, eps=1e-3)
    cfg["reflux"] = 0
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.burgers_sine(9) + 0.5)
    m0 = _mass(o)
    for _ in range(6):
        o.lt_step(0.5 * (1.0 / 512) / 1.6)
    assert abs(_mass(o)[0] - m0[0]) > 1e-9


def test_mass_conserved_diffusion_neumann_2d(oracle_mod):
    cfg = W.nagumo_2d(L=6, eps=1e-3, k=0.0)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.nagumo_front(6))
    m0 = _mass(o)
    for _ in range(3):
        o.lt_step(2e-6)
    assert abs(_mass(o)[0] - m0[0]) < 1e-15


def test_mass_energy_conserved_euler_sphere_3d(oracle_mod):
    # periodic, so that no boundary flux enters (at this coarse level the
    # discrete domain of dependence reaches the boundary within a step)
    cfg = W.euler_3d(L=4, eps=1e-3)
    cfg["bc"] = "periodic"
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.euler_sphere(4))
    m0 = _mass(o)
    for _ in range(2):
        ws = o.max_wavespeed()
        o.lt_step(W.euler_dt(cfg, ws, o.stats()["t"]) * 0.5)
    m1 = _mass(o)
    assert abs(m1[0] - m0[0]) < 1e-13 * abs(m0[0])
    assert abs(m1[4] - m0[4]) < 1e-13 * abs(m0[4])


# ---------------------------------------------------------------------------
# Table 1: self-convergence orders (Sec. 4.5)


def _gauss_avg(L):
    n = 1 << L
    xe = np.arange(n + 1) / n
    s = 10.0
    F = np.array([math.sqrt(math.pi) / (2 * s) * math.erf(s * (x - 0.25)) for x in xe])
    return (F[1:] - F[:-1]) * n


def _table1_run(oracle_mod, dt, uniform):
    cfg = dict(dim=1, L=9, l0=8, eps=0.0, pde="advection", adv_vel=[1.0, 0, 0],
               bc="periodic", recon=2, reflux=0, remesh=0)
    o = oracle_mod.Oracle(cfg)
    a9, a8 = _gauss_avg(9), _gauss_avg(8)
    if uniform:
        leaves = [(9, (i,)) for i in range(512)]
    else:
        leaves = [(9, (i,)) for i in range(256)] + [(8, (i,)) for i in range(128, 256)]
    leaves.sort(key=lambda lx: leaf_key(lx[0], 1, lx[1]))
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [(a9 if lev == 9 else a8)[x[0]]])
    o.set_leaves(keys, vals)
    n = int(round(1.0 / dt))
    for _ in range(n // 2):
        o.lt_step(dt)
    return o.reconstruct()[0]


def _order(oracle_mod, dt, uniform):
    q = [_table1_run(oracle_mod, dt / 2 ** j, uniform) for j in range(3)]
    return math.log2(np.abs(q[0] - q[1]).sum() / np.abs(q[1] - q[2]).sum())


def test_table1_fv_rk3_third_order(oracle_mod):
    gold = json.load(open(os.path.join(GOLDEN, "table1_orders.json")))
    p = _order(oracle_mod, gold["dt"][0], uniform=True)
    assert abs(p - gold["FV/RK3"][0]) < 0.05


def test_table1_mrlt_nerk3_second_order(oracle_mod):
    # the paper: MRLT/NERK3 converges with order 2 (third order is lost at the
    # level interface, eqs. EvRk3finer / EvRk3coarser).  The printed values
    # (1.7895, 1.9152) approach 2 from below; every reading of the paper's
    # open synchronisation choices scanned with tests/table1_readings.py
    # approaches it from above (2.01-2.94 at dt = 1.6e-4), so the pin is the
    # monotone approach to the limit order 2 over four halvings.
    p = [_order(oracle_mod, 1.6e-4 / 2 ** j, uniform=False) for j in range(3)]
    assert p[0] > p[1] > p[2] > 2.0
    assert abs(p[2] - 2.0) < 0.12
    assert abs(p[1] - 2.0) < 0.3


def test_table1_model_matches_oracle(oracle_mod):
    """The vectorised model of the Table 1 experiment used to scan the
    synchronisation readings takes the oracle's readings by default and
    gives its values bit for bit."""
    from tests.table1_readings import run
    dt = 1.6e-4
    cfg = dict(dim=1, L=9, l0=8, eps=0.0, pde="advection", adv_vel=[1.0, 0, 0],
               bc="periodic", recon=2, reflux=0, remesh=0)
    o = oracle_mod.Oracle(cfg)
    a9, a8 = _gauss_avg(9), _gauss_avg(8)
    leaves = [(9, (i,)) for i in range(256)] + [(8, (i,)) for i in range(128, 256)]
    leaves.sort(key=lambda lx: leaf_key(lx[0], 1, lx[1]))
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [(a9 if lev == 9 else a8)[x[0]]])
    o.set_leaves(keys, vals)
    for _ in range(60):
        o.lt_step(dt)
    assert np.array_equal(o.reconstruct()[0], run(dt, iters=120))


# ---------------------------------------------------------------------------
# exact solutions


def _burgers_to(oracle_mod, L, eps, nu, t):
    cfg = W.burgers_1d(L=L, eps=eps, nu=nu)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.burgers_sine(L))
    it = W.macro_iters(cfg)
    dx = 1.0 / (1 << L)
    dt_cfl = 0.4 / (1.0 / dx + 2 * nu / dx ** 2)
    nmac = math.ceil(t / (it * dt_cfl))
    for _ in range(nmac):
        o.lt_step(t / (nmac * it))
    return o.reconstruct()[0]


def test_heat_dirichlet_converges_to_closed_form(oracle_mod):
    """u_t = u_xx on [0,1], u = 0 at both ends, u0 = sin(pi x): the cell
    averages of exp(-pi^2 t) sin(pi x) are the exact solution.  The scheme
    is second order in space; a wrong boundary value (even instead of odd
    mirror, or a sign error) leaves an O(1) boundary error and no order."""
    t_end = 0.01
    errs = []
    for L in (5, 6, 7):
        cfg = W.linear_1d_dirichlet(L, eps=0.0)
        dx = 1.0 / (1 << L)
        it = W.macro_iters(cfg)
        nmac = math.ceil(t_end / (it * 0.25 * dx * dx / 2))
        dt = t_end / (nmac * it)
        o = oracle_mod.Oracle(cfg)
        o.load_finest(W.sine_half(L))
        for _ in range(nmac):
            o.lt_step(dt)
        got = o.reconstruct()[0]
        ex = W.sine_half(L)[0] * math.exp(-math.pi ** 2 * t_end)
        errs.append(np.abs(got - ex).mean())
    p1, p2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert errs[-1] < 2e-5, errs
    assert 1.7 < p1 < 2.4 and 1.7 < p2 < 2.4, (errs, p1, p2)
    # adaptive (eps = 1e-4): the thresholding error stays of the order of eps
    cfg = W.linear_1d_dirichlet(7, eps=1e-4)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.sine_half(7))
    it = W.macro_iters(cfg)
    nmac = math.ceil(t_end / (it * 0.25 / 128 ** 2 / 2))
    for _ in range(nmac):
        o.lt_step(t_end / (nmac * it))
    ex = W.sine_half(7)[0] * math.exp(-math.pi ** 2 * t_end)
    assert np.abs(o.reconstruct()[0] - ex).mean() < 1e-4


def test_dirichlet_changes_only_the_boundary_values(oracle_mod):
    """Dirichlet and Neumann runs of the same heat problem agree in the
    interior far from the walls after a short time, and differ next to
    them (the odd mirror pulls the wall cells towards zero)."""
    L = 7
    cfg_d = W.linear_1d_dirichlet(L, eps=0.0)
    cfg_n = dict(cfg_d, bc="neumann")
    q0 = np.ones((1, 1 << L))
    res = []
    for cfg in (cfg_d, cfg_n):
        o = oracle_mod.Oracle(cfg)
        o.load_finest(q0)
        o.lt_step(1e-6)
        res.append(o.reconstruct()[0])
    d, n = res
    assert np.array_equal(n, q0[0])                    # constant state under Neumann
    assert d[0] < 0.9 and d[-1] < 0.9                   # pulled down at the walls
    assert np.array_equal(d[20:-20], n[20:-20])        # untouched in the interior


def test_viscous_burgers_converges_to_cole_hopf(oracle_mod):
    # second-order convergence of the finite-volume operator to the exact
    # (Cole-Hopf) cell averages before the shock forms (t < 1/(2 pi))
    nu, t = 1e-3, 0.1
    errs = [np.abs(_burgers_to(oracle_mod, L, 0.0, nu, t) - X.cole_hopf_averages(L, t, nu)).mean()
            for L in (7, 8, 9)]
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert errs[2] < 5e-5, errs
    # the adaptive solve stays close to the exact solution
    ad = np.abs(_burgers_to(oracle_mod, 9, 1e-4, nu, t) - X.cole_hopf_averages(9, t, nu)).mean()
    assert ad < 5e-4, ad


def _sod(oracle_mod, L, eps, cfl, t=0.2):
    cfg = W.euler_1d(L=L, eps=eps)
    cfg["t_final"], cfg["cfl"] = t, cfl
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.euler_shock_tube(L))
    tt = 0.0
    while tt < t - 1e-14:
        o.lt_step(W.euler_dt(cfg, o.max_wavespeed(), tt))
        tt = o.stats()["t"]
    return o.reconstruct()[0]


def test_euler_shock_tube_converges_to_exact_riemann(oracle_mod):
    left, right, gamma, t = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, 0.2
    errs = [np.abs(_sod(oracle_mod, L, 0.0, 0.5) - X.riemann_cell_density(L, left, right, gamma, t)).mean()
            for L in (7, 8, 9)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 2.5e-3, errs
    # the local-time-stepping synchronisation error of the adaptive solve is
    # second order in time: it shrinks with the Courant number
    ex = X.riemann_cell_density(9, left, right, gamma, t)
    e_ad = [np.abs(_sod(oracle_mod, 9, 1e-3, c) - _sod(oracle_mod, 9, 0.0, c)).mean() for c in (0.5, 0.25, 0.1)]
    assert e_ad[0] > 2 * e_ad[1] > 4 * e_ad[2], e_ad
    assert np.abs(_sod(oracle_mod, 9, 1e-3, 0.25) - ex).mean() < 4e-3


def test_planar_3d_reduces_to_1d_exactly(oracle_mod):
    L = 5
    c1 = W.euler_1d(L=L, eps=1e-3)
    c3 = dict(W.euler_3d(L=L, eps=1e-3), lo=[0.0] * 3, hi=[1.0] * 3)
    for c in (c1, c3):
        c["thresh"] = 0
    q1 = W.euler_shock_tube(L)
    n = 1 << L
    q3 = np.zeros((5, n, n, n))
    q3[0] = q1[0][None, None, :]
    q3[1] = q1[1][None, None, :]
    q3[4] = q1[2][None, None, :]
    o1, o3 = oracle_mod.Oracle(c1), oracle_mod.Oracle(c3)
    o1.load_finest(q1)
    o3.load_finest(q3.reshape(5, -1))
    for _ in range(2):
        o1.lt_step(2e-3)
        o3.lt_step(2e-3)
    # same tree: every 1D leaf is a y-z layer of 3D leaves
    l1, l3 = o1.stats()["leaves"], o3.stats()["leaves"]
    assert all(l3[lev] == l1[lev] * 4 ** lev for lev in range(len(l1)))
    r1 = o1.reconstruct()
    r3 = o3.reconstruct().reshape(5, n, n, n)
    # values equal up to the summation order of the 2^d-child projections
    for k1, k3 in ((0, 0), (1, 1), (2, 4)):
        assert np.abs(r3[k3] - r1[k1][None, None, :]).max() < 1e-14
    assert not np.any(r3[2]) and not np.any(r3[3])


def test_spherical_3d_keeps_octahedral_symmetry(oracle_mod):
    cfg = W.euler_3d(L=4, eps=1e-3)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.euler_sphere(4))
    for _ in range(2):
        o.lt_step(W.euler_dt(cfg, o.max_wavespeed(), o.stats()["t"]))
    n = 16
    q = o.reconstruct().reshape(5, n, n, n)   # (k, z, y, x)
    rho, mx, my, mz, E = q
    tol = 1e-12
    # mirror x -> -x
    assert np.abs(rho - rho[:, :, ::-1]).max() < tol
    assert np.abs(mx + mx[:, :, ::-1]).max() < tol
    # swap x <-> y
    assert np.abs(rho - rho.transpose(0, 2, 1)).max() < tol
    assert np.abs(mx - my.transpose(0, 2, 1)).max() < tol
    # swap x <-> z
    assert np.abs(E - E.transpose(2, 1, 0)).max() < tol
    assert np.abs(mx - mz.transpose(2, 1, 0)).max() < tol
    assert rho.max() > rho.min() + 0.5
