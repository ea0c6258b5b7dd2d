"""Seeded synthetic workloads: problem configurations and initial cell averages.

This module holds no arithmetic of the multiresolution / local-time-stepping
method itself: it only describes problems (PDE, domain, boundary conditions,
levels, threshold) and integrates initial data into finest-level cell
averages.  Both the HIP path and the CPU oracle are fed from here.

Layout of every initial-data array: float64, shape (m, 2^{dL}), the finest
level in row-major order with x fastest (index x + n*(y + n*z)).
"""
from __future__ import annotations

import math

import numpy as np

SEED = 190508717

# ---------------------------------------------------------------------------
# configurations (plain dicts; each side converts them to its own struct)


def burgers_1d(L: int = 10, eps: float = 1e-3, l0: int = 2, nu: float = 1e-3) -> dict:
    """1D viscous Burgers, periodic [0,1], u0 = sin(2 pi x)."""
    return dict(name=f"burgers1d_L{L}", dim=1, L=L, l0=l0, eps=eps, pde="burgers", nu=nu,
                bc="periodic", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=1,
                reflux=1, remesh=1, t_final=0.5, cfl=0.5)


def nagumo_2d(L: int = 9, eps: float = 1e-3, l0: int = 2, k: float = 1e3, a: float = 0.2) -> dict:
    """2D Nagumo reaction-diffusion u_t = Lap u + k u (1-u)(u-a), Neumann unit square."""
    return dict(name=f"nagumo2d_L{L}", dim=2, L=L, l0=l0, eps=eps, pde="nagumo", nu=1.0,
                k_react=k, a_react=a, bc="neumann", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0],
                recon=1, thresh=1, reflux=1, remesh=1, t_final=0.01, cfl=0.5)


def euler_3d(L: int = 7, eps: float = 1e-3, l0: int = 2) -> dict:
    """3D Euler spherical Riemann problem on [-1,1]^3, Neumann."""
    return dict(name=f"euler3d_L{L}", dim=3, L=L, l0=l0, eps=eps, pde="euler", gamma=1.4,
                bc="neumann", lo=[-1.0, -1.0, -1.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=1,
                reflux=1, remesh=1, t_final=0.25, cfl=0.5)


def euler_2d(L: int = 8, eps: float = 1e-3, l0: int = 2) -> dict:
    """2D Euler four-quadrant Riemann problem on [0,1]^2, Neumann."""
    return dict(name=f"euler2d_L{L}", dim=2, L=L, l0=l0, eps=eps, pde="euler", gamma=1.4,
                bc="neumann", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=1,
                reflux=1, remesh=1, t_final=0.25, cfl=0.5)


def euler_1d(L: int = 9, eps: float = 1e-3, l0: int = 2) -> dict:
    """1D Euler shock tube on [0,1], Neumann."""
    return dict(name=f"euler1d_L{L}", dim=1, L=L, l0=l0, eps=eps, pde="euler", gamma=1.4,
                bc="neumann", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=1,
                reflux=1, remesh=1, t_final=0.2, cfl=0.5)


def burgers_2d(L: int = 9, eps: float = 1e-2, l0: int = 2) -> dict:
    """The paper's 2D inviscid Burgers problem (Sec. 5): Q_t + (Q^2/2)_x +
    (Q^2/2)_y = 0 on [0,1]^2, Q0 = sin(2 pi x) sin(2 pi y), homogeneous
    Dirichlet boundary, Courant number 0.5, fixed threshold eps = 0.01,
    t_f = 0.9."""
    return dict(name=f"burgers2d_L{L}", dim=2, L=L, l0=l0, eps=eps, pde="burgers", nu=0.0,
                bc="dirichlet", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=0,
                reflux=1, remesh=1, t_final=0.9, cfl=0.5)


def euler_laxliu6(L: int = 9, eps: float = 1e-2, l0: int = 2) -> dict:
    """The paper's 2D Euler problem (Sec. 5): Lax-Liu configuration 6 on
    [0,1]^2, Neumann, gamma = 1.4, Courant number 0.5, fixed threshold
    eps = 0.01, t_f = 0.25."""
    return dict(name=f"laxliu6_L{L}", dim=2, L=L, l0=l0, eps=eps, pde="euler", gamma=1.4,
                bc="neumann", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=0,
                reflux=1, remesh=1, t_final=0.25, cfl=0.5)


def linear_1d_dirichlet(L: int, eps: float = 0.0, l0: int = 2, nu: float = 1.0) -> dict:
    """Heat equation u_t = nu u_xx on [0,1] with u = 0 at both ends (test
    problem with a closed-form solution)."""
    return dict(name=f"heat1d_L{L}", dim=1, L=L, l0=l0, eps=eps, pde="linear", nu=nu, k_react=0.0,
                bc="dirichlet", lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], recon=1, thresh=1,
                reflux=1, remesh=1, t_final=0.01, cfl=0.25)


def flame_1d(L: int = 11, eps: float = 1e-2, l0: int = 2, flame_speed: int = -1) -> dict:
    """1D premixed flame of Sec. 5: T_t + v T_x = T_xx + omega(T) on (-15, 15),
    Ze = 10, tau = 0.8, dT/dx = 0 at x = -15, T = 0 at x = 15.  v = -v_f
    (flame_speed -1, the frame that moves with the front) or +v_f (+1, the
    sign as printed), v_f the integral of omega, per macro step."""
    return dict(name=f"flame1d_L{L}", dim=1, L=L, l0=l0, eps=eps, pde="flame", ze=10.0, tau=0.8,
                lewis=1.0, kappa=0.0, flame_speed=flame_speed, bc=[("neumann", "dirichlet"), "neumann", "neumann"],
                lo=[-15.0, 0.0, 0.0], hi=[15.0, 1.0, 1.0], adv_vel=[0.0, 0.0, 0.0], recon=1,
                thresh=1, reflux=1, remesh=1, t_final=5.0, cfl=0.5)


def flame_ball_3d(L: int = 7, eps: float = 1e-2, l0: int = 2, half_width: float = 15.0) -> dict:
    """3D flame ball of Sec. 5: T and Y with Lewis number 0.3 and radiation
    kappa = 0.1, Ze = 10, tau = 0.64, Neumann; the box (-15, 15)^3 (the
    paper does not state it; the 1D flame's interval on every axis)."""
    w = half_width
    return dict(name=f"flameball3d_L{L}", dim=3, L=L, l0=l0, eps=eps, pde="flameball", ze=10.0,
                tau=0.64, lewis=0.3, kappa=0.1, flame_speed=0, bc="neumann", lo=[-w, -w, -w],
                hi=[w, w, w], adv_vel=[0.0, 0.0, 0.0], recon=1, thresh=1, reflux=1, remesh=1,
                t_final=5.0, cfl=0.1)


def ncomp(cfg: dict) -> int:
    if cfg["pde"] == "euler":
        return cfg["dim"] + 2
    return 2 if cfg["pde"] == "flameball" else 1


# ---------------------------------------------------------------------------
# time step rules (the caller of a macro step chooses dt_L)


def macro_iters(cfg: dict) -> int:
    return 1 << (cfg["L"] - cfg.get("l0", 2))


def burgers_dt(cfg: dict, umax: float = 1.0) -> float:
    """dt_L for a Burgers configuration: CFL sigma on the finest level (rate
    d |u|max / dx plus the diffusive term), rounded so that t_final is
    reached after a whole number of macro steps."""
    dx = 1.0 / (1 << cfg["L"])
    dt_cfl = cfg["cfl"] / (cfg["dim"] * umax / dx + 2 * cfg["dim"] * cfg["nu"] / dx ** 2)
    it = macro_iters(cfg)
    nmac = math.ceil(cfg["t_final"] / (it * dt_cfl))
    return cfg["t_final"] / (nmac * it)


def nagumo_dt(cfg: dict) -> float:
    """dt_L for the Nagumo configuration: sigma / (2d/dx^2 + 0.8 k), rounded to
    a whole number of macro steps up to t_final."""
    dx = 1.0 / (1 << cfg["L"])
    dt_cfl = cfg["cfl"] / (2 * cfg["dim"] / dx ** 2 + 0.8 * cfg["k_react"])
    it = macro_iters(cfg)
    nmac = math.ceil(cfg["t_final"] / (it * dt_cfl))
    return cfg["t_final"] / (nmac * it)


def flame_dt(cfg: dict, vmax: float = 1.5) -> float:
    """dt_L for the flame problems: Courant number sigma on the finest level
    for the fastest diffusion (coefficient max(1, 1/Le)) plus advection at
    speed vmax; and the coarsest level's local step 2^{L-l0} dt_L within the
    RK3 stability interval of the burnt-gas relaxation, whose rate is
    Ze^2 / (2 Le) (it binds only on coarse finest levels, never at the
    paper's L); rounded to a whole number of macro steps up to t_final."""
    dx = (cfg["hi"][0] - cfg["lo"][0]) / (1 << cfg["L"])
    le = cfg.get("lewis", 1.0)
    dmax = max(1.0, 1.0 / le)
    vel = vmax if cfg.get("flame_speed", 0) else sum(abs(v) for v in cfg["adv_vel"][:cfg["dim"]])
    it = macro_iters(cfg)
    dt_cfl = cfg["cfl"] / (2 * cfg["dim"] * dmax / dx ** 2 + vel / dx)
    dt_src = 2.0 / (cfg["ze"] ** 2 / (2 * le) * (it if cfg.get("lt", 1) else 1))
    dt_cfl = min(dt_cfl, dt_src)
    nmac = math.ceil(cfg["t_final"] / (it * dt_cfl))
    return cfg["t_final"] / (nmac * it)


def euler_dt(cfg: dict, max_wavespeed: float, t: float) -> float:
    dx = (cfg["hi"][0] - cfg["lo"][0]) / (1 << cfg["L"])
    it = macro_iters(cfg)
    return min(cfg["cfl"] * dx / max_wavespeed, (cfg["t_final"] - t) / it)


# ---------------------------------------------------------------------------
# initial cell averages

_GL4 = np.polynomial.legendre.leggauss(4)


def _centers(n: int, lo: float, hi: float):
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx, dx


def burgers_sine(L: int, phase: float = 0.0) -> np.ndarray:
    """Exact cell averages of sin(2 pi (x + phase)) on [0,1]."""
    n = 1 << L
    xe = np.arange(n + 1) / n + phase
    avg = (np.cos(2 * np.pi * xe[:-1]) - np.cos(2 * np.pi * xe[1:])) * (n / (2 * np.pi))
    return avg.reshape(1, n)


def burgers_modes(L: int, seed: int) -> np.ndarray:
    """Exact cell averages of sum_m a_m sin(2 pi m x + phi_m) / sum a_m, m = 1..4."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, 4)
    ph = rng.uniform(0.0, 2 * np.pi, 4)
    n = 1 << L
    xe = np.arange(n + 1) / n
    avg = np.zeros(n)
    for mm in range(1, 5):
        prim = -np.cos(2 * np.pi * mm * xe + ph[mm - 1]) / (2 * np.pi * mm)
        avg += a[mm - 1] * (prim[1:] - prim[:-1]) * n
    return (avg / a.sum()).reshape(1, n)


def nagumo_front(L: int, seed: int = SEED, width: float = 0.02, amp: float = 0.05) -> np.ndarray:
    """u0 = (1 - tanh((x - 0.25 - eta(y)) / width)) / 2 with
    eta(y) = amp * sum_{m=1..8} c_m cos(m pi y) / sum |c_m|, c_m ~ U(-1,1)
    seeded; 4x4 Gauss-Legendre cell averages on [0,1]^2."""
    rng = np.random.default_rng(seed)
    cm = rng.uniform(-1.0, 1.0, 8)
    n = 1 << L
    xc, dx = _centers(n, 0.0, 1.0)
    g, w = _GL4
    xs = (xc[:, None] + 0.5 * dx * g[None, :])  # (n, 4)
    eta = np.zeros_like(xs)
    for mm in range(1, 9):
        eta += cm[mm - 1] * np.cos(mm * np.pi * xs)
    eta *= amp / np.abs(cm).sum()
    # u(x, y): x points (n,4) along axis x; y points (n,4) give eta
    X = xs[None, None, :, :]          # (1,1,nx,4)
    E = eta[:, :, None, None]         # (ny,4,1,1)
    U = 0.5 * (1.0 - np.tanh((X - 0.25 - E) / width))
    avg = np.einsum("yjxi,j,i->yx", U, w, w) * 0.25
    return avg.reshape(1, n * n)


def burgers_sinsin(L: int) -> np.ndarray:
    """Exact cell averages of sin(2 pi x) sin(2 pi y) on [0,1]^2 (a product
    of the 1D averages)."""
    a = burgers_sine(L)[0]
    n = 1 << L
    return np.outer(a, a).reshape(1, n * n)


def sine_half(L: int) -> np.ndarray:
    """Exact cell averages of sin(pi x) on [0,1]."""
    n = 1 << L
    xe = np.arange(n + 1) / n
    return ((np.cos(np.pi * xe[:-1]) - np.cos(np.pi * xe[1:])) * (n / np.pi)).reshape(1, n)


# Lax-Liu configuration 6: (rho, u, v, p) of quadrants 1..4 (the paper's
# table of initial conditions for the 2D Euler equations)
LAXLIU6 = ((1.0, 0.75, -0.5, 1.0), (2.0, 0.75, 0.5, 1.0), (1.0, -0.75, 0.5, 1.0), (3.0, -0.75, -0.5, 1.0))


def euler_state(rho, u, v, w, p, gamma=1.4, dim=3):
    vel = [u, v, w][:dim]
    E = p / (gamma - 1.0) + 0.5 * rho * sum(x * x for x in vel)
    return [rho] + [rho * x for x in vel] + [E]


def euler_sphere(L: int, gamma: float = 1.4, radius: float = 0.4) -> np.ndarray:
    """Spherical Riemann problem on [-1,1]^3: rho=1, p=1 inside r < radius,
    rho=0.125, p=0.1 outside, zero velocity; 4^3 Gauss-Legendre averages."""
    n = 1 << L
    xc, dx = _centers(n, -1.0, 1.0)
    g, w = _GL4
    pts = xc[:, None] + 0.5 * dx * g[None, :]   # (n,4)
    ww = w * 0.5
    inside = np.zeros((n, n, n))
    r2x = pts ** 2
    for a in range(4):
        for b in range(4):
            for c in range(4):
                r2 = r2x[None, None, :, a] + r2x[None, :, None, b] + r2x[:, None, None, c]
                inside += ww[a] * ww[b] * ww[c] * (r2 < radius * radius)
    fin = euler_state(1.0, 0, 0, 0, 1.0, gamma)
    fout = euler_state(0.125, 0, 0, 0, 0.1, gamma)
    q = np.zeros((5, n ** 3))
    fr = inside.reshape(-1)
    for k in range(5):
        q[k] = fr * fin[k] + (1 - fr) * fout[k]
    return q


def euler_quadrants(L: int, states, gamma: float = 1.4) -> np.ndarray:
    """Four-quadrant Riemann problem on [0,1]^2.  states[j] = (rho, u, v, p)
    for quadrants 1..4 = [.5,1]x[.5,1], [0,.5]x[.5,1], [0,.5]x[0,.5],
    [.5,1]x[0,.5].  Faces align with x = y = 0.5, so the averages are exact."""
    n = 1 << L
    h = n // 2
    q = np.zeros((4, n, n))
    quad = {(1, 1): 0, (0, 1): 1, (0, 0): 2, (1, 0): 3}
    for (qx, qy), j in quad.items():
        rho, u, v, p = states[j]
        cons = euler_state(rho, u, v, 0.0, p, gamma, dim=2)
        for k in range(4):
            q[k, qy * h:(qy + 1) * h, qx * h:(qx + 1) * h] = cons[k]
    return q.reshape(4, n * n)


def euler_quadrants_seeded(L: int, seed: int, gamma: float = 1.4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 2.0)
        p = rng.uniform(0.1, 2.0)
        u, v = rng.uniform(-0.8, 0.8, 2)
        states.append((rho, u, v, p))
    return euler_quadrants(L, states, gamma)


def euler_shock_tube(L: int, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x0: float = 0.5,
                     gamma: float = 1.4) -> np.ndarray:
    """1D shock tube (rho, u, p) on [0,1] with the jump on a cell face."""
    n = 1 << L
    q = np.zeros((3, n))
    j = int(round(x0 * n))
    for sl, st in ((slice(0, j), left), (slice(j, n), right)):
        cons = euler_state(st[0], st[1], 0, 0, st[2], gamma, dim=1)
        for k in range(3):
            q[k, sl] = cons[k]
    return q


def flame_front(L: int, lo: float = -15.0, hi: float = 15.0, x0: float = 1.0) -> np.ndarray:
    """Sec. 5 one-dimensional flame: T = 1 for x <= x0, exp(x0 - x) beyond;
    exact cell averages."""
    n = 1 << L
    dx = (hi - lo) / n
    a = lo + dx * np.arange(n)
    b = a + dx
    burnt = np.clip(np.minimum(b, x0) - a, 0.0, None)            # part with x <= x0
    s = np.maximum(a, x0)
    fresh = np.where(b > x0, np.exp(x0 - s) - np.exp(x0 - b), 0.0)
    return ((burnt + fresh) / dx).reshape(1, n)


def flame_ball(L: int, lo: float = -15.0, hi: float = 15.0, lewis: float = 0.3, r0: float = 1.0,
               axes=(1.5, 1.5, 3.0), theta: float = math.pi / 3, phi: float = math.pi / 4) -> np.ndarray:
    """Sec. 5 three-dimensional flame ball: ellipsoidal radius r of the
    rotated coordinates; T = 1, Y = 0 for r <= r0, else T = exp(1 - r/r0),
    Y = 1 - exp(Le (1 - r/r0)); 4^3 Gauss-Legendre averages."""
    n = 1 << L
    xc, dx = _centers(n, lo, hi)
    g, w = _GL4
    pts = xc[:, None] + 0.5 * dx * g[None, :]   # (n,4)
    ww = w * 0.5
    ct, st, cp, sp = math.cos(theta), math.sin(theta), math.cos(phi), math.sin(phi)
    T = np.zeros((n, n, n))
    Y = np.zeros((n, n, n))
    for a in range(4):
        x = pts[None, None, :, a]
        for b in range(4):
            y = pts[None, :, None, b]
            for c in range(4):
                z = pts[:, None, None, c]
                X1 = x * ct - y * st
                u = x * st + y * ct
                Y1 = u * cp - z * sp
                Z1 = u * sp + z * cp
                r = np.sqrt((X1 / axes[0]) ** 2 + (Y1 / axes[1]) ** 2 + (Z1 / axes[2]) ** 2)
                out = r > r0
                wt = ww[a] * ww[b] * ww[c]
                T += wt * np.where(out, np.exp(1.0 - r / r0), 1.0)
                Y += wt * np.where(out, 1.0 - np.exp(lewis * (1.0 - r / r0)), 0.0)
    return np.stack([T.reshape(-1), Y.reshape(-1)])


def initial_data(cfg: dict, seed: int = SEED) -> np.ndarray:
    name = cfg["pde"]
    if cfg.get("name", "").startswith("burgers2d"):
        return burgers_sinsin(cfg["L"])
    if cfg.get("name", "").startswith("laxliu6"):
        return euler_quadrants(cfg["L"], LAXLIU6, cfg.get("gamma", 1.4))
    if name == "burgers":
        return burgers_sine(cfg["L"])
    if name == "nagumo":
        return nagumo_front(cfg["L"], seed)
    if name == "flame":
        return flame_front(cfg["L"], cfg["lo"][0], cfg["hi"][0])
    if name == "flameball":
        return flame_ball(cfg["L"], cfg["lo"][0], cfg["hi"][0], cfg.get("lewis", 0.3))
    if name == "euler" and cfg["dim"] == 3:
        return euler_sphere(cfg["L"], cfg.get("gamma", 1.4))
    if name == "euler" and cfg["dim"] == 2:
        return euler_quadrants_seeded(cfg["L"], seed, cfg.get("gamma", 1.4))
    if name == "euler" and cfg["dim"] == 1:
        return euler_shock_tube(cfg["L"])
    raise ValueError(f"no initial data for {name}")
