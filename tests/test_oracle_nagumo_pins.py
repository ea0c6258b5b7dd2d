"""Pins of the oracle's Nagumo reaction-diffusion problem by what the
mathematics fixes, independent of any second implementation of the source.

* A spatially uniform state feels no diffusive flux, so on a multilevel
  tree every leaf follows the scalar ODE u' = k u (1 - u)(u - a) with the
  compact RK3 step of its own level (local time stepping: 2^{L-l} dt_L).
  The leaves are compared with scipy's integrator; the deviation must be
  small and fall when dt is halved (a wrong sign, factor or root in the
  source gives an O(1) deviation that does not fall).
* The travelling wave of u_t = u_xx + k u (1 - u)(u - a) with 0 < a < 1/2
  is u = 1 / (1 + exp(sqrt(k/2) (x - c t))) with speed
  c = sqrt(k/2) (1 - 2a) (about 13.42 at k = 1e3, a = 0.2): the adaptive
  1D solve started from that profile must carry its u = 1/2 point at c.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp

from paper_1905_08717_amd import workloads as W
from tests.trees import build_tree, leaf_arrays

K, A = 1.0e3, 0.2


def _ode(u0, t):
    sol = solve_ivp(lambda _t, u: K * u * (1.0 - u) * (u - A), (0.0, t), [u0],
                    method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[0, -1]


def _uniform_run(oracle_mod, u0, dt, nmac):
    cfg = dict(W.nagumo_2d(L=6, eps=0.0), dim=1, remesh=0)
    # graded 1D tree with leaves on every level 2..6
    leaves = build_tree(1, 6, 2, lambda c: 2 + int(4 * c[0] + 1e-12) + (1 if c[0] > 0.9 else 0))
    keys, vals = leaf_arrays(1, leaves, lambda lev, x: [u0])
    o = oracle_mod.Oracle(cfg)
    o.set_leaves(keys, vals)
    for _ in range(nmac):
        o.lt_step(dt)
    k2, q = o.get_leaves()
    lev = (k2 >> np.uint64(56)).astype(int)
    return lev, q[0]


def test_uniform_state_follows_the_source_ode(oracle_mod):
    u0 = 0.3                     # above a: grows towards the stable state 1
    t_end = 8.0e-3               # u: 0.3 -> 0.81 through the steep part
    it = 1 << (6 - 2)            # fine iterations per macro step
    errs = []
    for nmac in (40, 80):
        dt = t_end / (nmac * it)
        lev, u = _uniform_run(oracle_mod, u0, dt, nmac)
        assert set(lev.tolist()) == {2, 3, 4, 5, 6}
        exact = _ode(u0, t_end)
        assert 0.6 < exact < 0.99
        errs.append(np.abs(u - exact).max())
    # every leaf within 1e-5 of the ODE (the coarsest leaves step 16 dt_L);
    # the deviation falls at least like dt^1.8 (RK3 in each leaf plus the
    # second-order level synchronisation, whose differences feel diffusion)
    assert errs[0] < 1e-5
    assert errs[0] / errs[1] > 3.5


def test_wrong_source_sign_is_detected(oracle_mod):
    """The ODE comparison above separates the printed source from the one
    with the sign of (u - a) flipped (the two trajectories leave u0 = 0.3
    in opposite directions)."""
    lev, u = _uniform_run(oracle_mod, 0.3, 8.0e-3 / (40 * 16), 40)
    flipped = solve_ivp(lambda _t, v: K * v * (1.0 - v) * (A - v), (0.0, 8.0e-3), [0.3],
                        method="DOP853", rtol=1e-13, atol=1e-15).y[0, -1]
    assert np.abs(u - flipped).min() > 0.2


def test_travelling_front_speed(oracle_mod):
    L = 10
    cfg = dict(W.nagumo_2d(L=L, eps=1e-3), dim=1)
    s = math.sqrt(K / 2.0)
    c_exact = s * (1.0 - 2.0 * A)
    n = 1 << L
    xe = np.arange(n + 1) / n
    # exact cell averages of 1 / (1 + exp(s (x - x0))): primitive -log(1 + exp(-s(x - x0)))/s
    x0 = 0.3

    def prim(x):
        z = s * (x - x0)
        return x - np.logaddexp(0.0, z) / s

    u0 = (prim(xe[1:]) - prim(xe[:-1])) * n
    o = oracle_mod.Oracle(cfg)
    o.load_finest(u0[None, :])
    dt = W.nagumo_dt(dict(cfg, t_final=0.02))
    it = W.macro_iters(cfg)

    def front(q):
        i = int(np.argmax(q < 0.5))
        xc = (np.arange(n) + 0.5) / n
        return xc[i - 1] + (xc[i] - xc[i - 1]) * (q[i - 1] - 0.5) / (q[i - 1] - q[i])

    nmac = int(round(0.02 / (dt * it)))
    # let the profile settle for a quarter of the run, then time the front
    m0 = nmac // 4
    for _ in range(m0):
        o.lt_step(dt)
    xa, ta = front(o.reconstruct()[0]), m0 * it * dt
    for _ in range(nmac - m0):
        o.lt_step(dt)
    xb, tb = front(o.reconstruct()[0]), nmac * it * dt
    c = (xb - xa) / (tb - ta)
    assert abs(c / c_exact - 1.0) < 0.01, (c, c_exact)      # measured: 0.04 %
    st = o.stats()
    # an adapted tree: about 100 leaves on four levels instead of 1024 cells
    assert sum(st["leaves"]) < n // 4 and sum(1 for v in st["leaves"] if v) >= 3
