"""The seeded input generators (shared by the HIP path and the oracle)."""
import numpy as np

from paper_1905_08717_amd import workloads as W


def test_burgers_sine_exact_averages():
    q = W.burgers_sine(10)
    assert q.shape == (1, 1024)
    assert abs(q.sum()) < 1e-12
    # average over a cell of sin tends to the midpoint value
    x = (np.arange(1024) + 0.5) / 1024
    assert np.abs(q[0] - np.sin(2 * np.pi * x)).max() < 2e-6


def test_nagumo_front_seeded_and_bounded():
    a = W.nagumo_front(7, seed=W.SEED)
    b = W.nagumo_front(7, seed=W.SEED)
    c = W.nagumo_front(7, seed=W.SEED + 1)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() <= 1.0
    g = a.reshape(128, 128)            # (y, x)
    assert g[:, 0].min() > 0.99 and g[:, -1].max() < 1e-6


def test_euler_sphere_states():
    q = W.euler_sphere(4)
    assert q.shape == (5, 4096)
    assert np.isclose(q[0].max(), 1.0) and np.isclose(q[0].min(), 0.125)
    assert not np.any(q[1:4])


def test_euler_quadrants_seeded_ranges():
    q = W.euler_quadrants_seeded(6, W.SEED + 3)
    rho = q[0]
    assert rho.min() >= 0.1 and rho.max() <= 2.0
    assert len(np.unique(rho)) <= 4


def test_time_step_rules_hit_t_final():
    cfg = W.burgers_1d()
    dt = W.burgers_dt(cfg)
    n = cfg["t_final"] / (dt * W.macro_iters(cfg))
    assert abs(n - round(n)) < 1e-9 and round(n) == 13
    cfg2 = W.nagumo_2d()
    dt2 = W.nagumo_dt(cfg2)
    n2 = cfg2["t_final"] / (dt2 * W.macro_iters(cfg2))
    assert abs(n2 - round(n2)) < 1e-9 and round(n2) == 164
