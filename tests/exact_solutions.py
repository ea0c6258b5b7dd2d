"""Exact solutions used to pin the oracle (test helpers).

* Cole-Hopf solution of viscous Burgers u_t + (u^2/2)_x = nu u_xx on the
  periodic unit interval with u0 = sin(2 pi x): u = -2 nu (log phi)_x with
  phi the heat-kernel convolution of exp(-Psi/(2 nu)), Psi' = u0.  Exact cell
  averages follow from differences of log phi at the faces.
* The exact Riemann solver of the 1D Euler equations for an ideal gas
  (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4):
  Newton iteration for the star pressure, then sampling of the wave fan.
"""
from __future__ import annotations

import math

import numpy as np


def _logsumexp(a, axis=-1):
    m = a.max(axis=axis, keepdims=True)
    return (m + np.log(np.exp(a - m).sum(axis=axis, keepdims=True))).squeeze(axis)


def cole_hopf_log_phi(x: np.ndarray, t: float, nu: float) -> np.ndarray:
    sig = math.sqrt(2.0 * nu * t)
    s = np.linspace(-14.0 * sig, 14.0 * sig, 4001)
    dy = s[1] - s[0]
    y = x[:, None] + s[None, :]
    psi = (1.0 - np.cos(2.0 * np.pi * y)) / (2.0 * np.pi)
    expo = -(s[None, :] ** 2) / (4.0 * nu * t) - psi / (2.0 * nu)
    return _logsumexp(expo) + math.log(dy)


def cole_hopf_averages(L: int, t: float, nu: float) -> np.ndarray:
    n = 1 << L
    xf = np.arange(n + 1) / n
    lp = cole_hopf_log_phi(xf, t, nu)
    return -2.0 * nu * (lp[1:] - lp[:-1]) * n


def riemann_exact(left, right, gamma, xi):
    """Sample the exact solution (rho, u, p) of the Riemann problem at x/t = xi."""
    rl, ul, pl = left
    rr, ur, pr = right
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (2.0 * gamma)
    g2 = (gamma + 1.0) / (2.0 * gamma)

    def fk(p, rk, pk, ak):
        if p > pk:
            A = 2.0 / ((gamma + 1.0) * rk)
            B = (gamma - 1.0) / (gamma + 1.0) * pk
            q = math.sqrt(A / (p + B))
            return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
        r = p / pk
        return 2.0 * ak / (gamma - 1.0) * (r ** g1 - 1.0), 1.0 / (rk * ak) * r ** (-g2)

    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, al)
        f2, d2 = fk(p, rr, pr, ar)
        f = f1 + f2 + (ur - ul)
        pn = max(1e-12, p - f / (d1 + d2))
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    f1, _ = fk(p, rl, pl, al)
    f2, _ = fk(p, rr, pr, ar)
    um = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    pm = p
    out = np.zeros((3, len(xi)))
    gm = gamma
    for j, s in enumerate(xi):
        if s <= um:
            if pm > pl:
                sl = ul - al * math.sqrt(g2 * pm / pl + g1)
                if s <= sl:
                    out[:, j] = (rl, ul, pl)
                else:
                    r = rl * ((pm / pl + (gm - 1) / (gm + 1)) / ((gm - 1) / (gm + 1) * pm / pl + 1))
                    out[:, j] = (r, um, pm)
            else:
                shl = ul - al
                if s <= shl:
                    out[:, j] = (rl, ul, pl)
                else:
                    cml = al * (pm / pl) ** g1
                    stl = um - cml
                    if s > stl:
                        out[:, j] = (rl * (pm / pl) ** (1 / gm), um, pm)
                    else:
                        u = 2 / (gm + 1) * (al + (gm - 1) / 2 * ul + s)
                        c = 2 / (gm + 1) * (al + (gm - 1) / 2 * (ul - s))
                        r = rl * (c / al) ** (2 / (gm - 1))
                        out[:, j] = (r, u, pl * (c / al) ** (2 * gm / (gm - 1)))
        else:
            if pm > pr:
                sr = ur + ar * math.sqrt(g2 * pm / pr + g1)
                if s >= sr:
                    out[:, j] = (rr, ur, pr)
                else:
                    r = rr * ((pm / pr + (gm - 1) / (gm + 1)) / ((gm - 1) / (gm + 1) * pm / pr + 1))
                    out[:, j] = (r, um, pm)
            else:
                shr = ur + ar
                if s >= shr:
                    out[:, j] = (rr, ur, pr)
                else:
                    cmr = ar * (pm / pr) ** g1
                    str_ = um + cmr
                    if s <= str_:
                        out[:, j] = (rr * (pm / pr) ** (1 / gm), um, pm)
                    else:
                        u = 2 / (gm + 1) * (-ar + (gm - 1) / 2 * ur + s)
                        c = 2 / (gm + 1) * (ar - (gm - 1) / 2 * (ur - s))
                        r = rr * (c / ar) ** (2 / (gm - 1))
                        out[:, j] = (r, u, pr * (c / ar) ** (2 * gm / (gm - 1)))
    return out


def riemann_cell_density(L, left, right, gamma, t, x0=0.5, sub=16):
    n = 1 << L
    xs = (np.arange(n * sub) + 0.5) / (n * sub)
    w = riemann_exact(left, right, gamma, (xs - x0) / t)
    return w[0].reshape(n, sub).mean(axis=1)
