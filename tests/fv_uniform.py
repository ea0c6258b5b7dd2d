"""Uniform-grid finite-volume / compact RK3 reference in numpy (test helper).

An independent, much simpler scheme than the oracle: one uniform level, no
tree, no local time stepping, no synchronisation.  With eps = 0 the MRLT
macro step must reduce to exactly this (same expression trees, so the
comparison is bit for bit).  Written from the finite-volume form
dq/dt = -(F_{i+1/2} - F_{i-1/2})/dx + S (Sec. 2) and the compact RK3 of
Sec. 3, with the flux readings of the oracle (MUSCL-minmod, Godunov for
Burgers, AUSM+ for Euler).
"""
from __future__ import annotations

import numpy as np


def _pad(q: np.ndarray, axis: int, bc: str) -> np.ndarray:
    width = [(0, 0)] * q.ndim
    width[axis] = (2, 2)
    if bc == "dirichlet":
        # homogeneous Dirichlet: mirrored cells with the opposite sign
        P = np.pad(q, width, mode="symmetric")
        idx = [slice(None)] * q.ndim
        for sl in (slice(0, 2), slice(-2, None)):
            idx[axis] = sl
            P[tuple(idx)] = -P[tuple(idx)]
        return P
    return np.pad(q, width, mode="wrap" if bc == "periodic" else "symmetric")


def _minmod(a, b):
    return np.where((a > 0) & (b > 0), np.minimum(a, b),
                    np.where((a < 0) & (b < 0), np.maximum(a, b), 0.0))


def _recon(mode, c0, c1, c2, c3):
    if mode == 1:
        sl = _minmod(c1 - c0, c2 - c1)
        sr = _minmod(c2 - c1, c3 - c2)
        return c1 + 0.5 * sl, c2 - 0.5 * sr
    return c1, c2


def _mplus(M):
    t = M + 1.0
    q = (M * M) - 1.0
    return np.where(np.abs(M) < 1.0, (0.25 * (t * t)) + (0.125 * (q * q)), 0.5 * (M + np.abs(M)))


def _mminus(M):
    t = M - 1.0
    q = (M * M) - 1.0
    return np.where(np.abs(M) < 1.0, (-(0.25 * (t * t))) - (0.125 * (q * q)), 0.5 * (M - np.abs(M)))


def _pplus(M):
    t = M + 1.0
    q = (M * M) - 1.0
    return np.where(np.abs(M) < 1.0, ((0.25 * (t * t)) * (2.0 - M)) + ((0.1875 * M) * (q * q)),
                    np.where(M > 0.0, 1.0, 0.0))


def _pminus(M):
    t = M - 1.0
    q = (M * M) - 1.0
    return np.where(np.abs(M) < 1.0, ((0.25 * (t * t)) * (2.0 + M)) - ((0.1875 * M) * (q * q)),
                    np.where(M < 0.0, 1.0, 0.0))


def _prim(d, gm1, q):
    rho = q[0]
    w = [rho]
    kin = None
    for i in range(d):
        u = q[1 + i] / rho
        w.append(u)
        kin = (u * u) if i == 0 else (kin + (u * u))
    w.append(gm1 * (q[d + 1] - ((0.5 * rho) * kin)))
    return w


def _ausm(d, ax, gamma, wl, wr):
    gm1 = gamma - 1.0
    rl, pl, rr, pr = wl[0], wl[d + 1], wr[0], wr[d + 1]
    al = np.sqrt((gamma * pl) / rl)
    ar = np.sqrt((gamma * pr) / rr)
    ah = 0.5 * (al + ar)
    ml = wl[1 + ax] / ah
    mr = wr[1 + ax] / ah
    mh = _mplus(ml) + _mminus(mr)
    ph = (_pplus(ml) * pl) + (_pminus(mr) * pr)
    mp = 0.5 * (mh + np.abs(mh))
    mm = 0.5 * (mh - np.abs(mh))
    kl = kr = None
    for i in range(d):
        kl = (wl[1] * wl[1]) if i == 0 else (kl + (wl[1 + i] * wl[1 + i]))
        kr = (wr[1] * wr[1]) if i == 0 else (kr + (wr[1 + i] * wr[1 + i]))
    hl = ((pl / gm1) + ((0.5 * rl) * kl)) + pl
    hr = ((pr / gm1) + ((0.5 * rr) * kr)) + pr
    F = [ah * ((mp * rl) + (mm * rr))]
    for i in range(d):
        F.append(ah * ((mp * (rl * wl[1 + i])) + (mm * (rr * wr[1 + i]))))
    F[1 + ax] = F[1 + ax] + ph
    F.append(ah * ((mp * hl) + (mm * hr)))
    return F


def _faces(cfg, q, axis_q, ax, invdx):
    """Fluxes on the n+1 faces along array axis axis_q (spatial direction ax)."""
    pde = cfg["pde"]
    bc = cfg.get("bc", "periodic")
    bc = bc[ax] if isinstance(bc, (list, tuple)) else bc
    P = _pad(q, axis_q, bc)
    n = q.shape[axis_q]

    def sl(j):
        idx = [slice(None)] * P.ndim
        idx[axis_q] = slice(j, j + n + 1)
        return P[tuple(idx)]

    c = [sl(j) for j in range(4)]
    recon = cfg.get("recon", 1)
    if pde == "burgers":
        uL, uR = _recon(recon, c[0][0], c[1][0], c[2][0], c[3][0])
        a = np.where(uL > 0.0, uL, 0.0)
        b = np.where(uR < 0.0, uR, 0.0)
        fa = 0.5 * (a * a)
        fb = 0.5 * (b * b)
        nudx = cfg["nu"] * invdx
        return [np.where(fa > fb, fa, fb) - (nudx * (c[2][0] - c[1][0]))]
    if pde in ("nagumo", "linear"):
        nudx = cfg["nu"] * invdx
        return [-(nudx * (c[2][0] - c[1][0]))]
    if pde == "advection":
        vel = cfg["adv_vel"][ax]
        if recon == 2:
            return [vel * (0.5 * (c[1][0] + c[2][0]))]
        qL, qR = _recon(recon, c[0][0], c[1][0], c[2][0], c[3][0])
        return [vel * qL if vel >= 0.0 else vel * qR]
    if pde == "euler":
        d = cfg["dim"]
        gamma = cfg.get("gamma", 1.4)
        w = [_prim(d, gamma - 1.0, [cj[k] for k in range(d + 2)]) for cj in c]
        wl, wr = [], []
        for k in range(d + 2):
            l, r = _recon(recon, w[0][k], w[1][k], w[2][k], w[3][k])
            wl.append(l)
            wr.append(r)
        return _ausm(d, ax, gamma, wl, wr)
    raise ValueError(pde)


def rhs(cfg, q, level):
    """q: (m, n, ..., n) array with x the LAST axis.  Returns R of the same shape."""
    d = cfg["dim"]
    m = q.shape[0]
    R = None
    for ax in range(d):
        axis_q = q.ndim - 1 - ax            # x is the last axis
        n = q.shape[axis_q]
        dx = (cfg.get("hi", [1.0] * 3)[ax] - cfg.get("lo", [0.0] * 3)[ax]) / n
        invdx = 1.0 / dx
        F = _faces(cfg, q, axis_q, ax, invdx)
        for k in range(m):
            Fk = np.asarray(F[k])
            idx_m = [slice(None)] * Fk.ndim
            idx_p = [slice(None)] * Fk.ndim
            idx_m[axis_q - 1] = slice(0, n)
            idx_p[axis_q - 1] = slice(1, n + 1)
            r = (Fk[tuple(idx_m)] - Fk[tuple(idx_p)]) * invdx
            if R is None:
                R = [None] * m
            R[k] = r if ax == 0 else (R[k] + r)
    R = np.array(R)
    if cfg["pde"] == "nagumo":
        u = q[0]
        R[0] = R[0] + (((cfg["k_react"] * u) * (1.0 - u)) * (u - cfg["a_react"]))
    elif cfg["pde"] == "linear":
        R[0] = R[0] + (cfg["k_react"] * q[0])
    return R


def rk3_step(cfg, q, level, h):
    """One compact RK3 step (Sec. 3) of size h."""
    R1 = rhs(cfg, q, level)
    q1 = q + (h * R1)
    R2 = rhs(cfg, q1, level)
    qh = ((0.75 * q) + (0.25 * q1)) + ((0.25 * h) * R2)
    R3 = rhs(cfg, qh, level)
    return ((1.0 / 3.0) * q + (2.0 / 3.0) * qh) + (((2.0 / 3.0) * h) * R3)


def to_grid(cfg, q_flat, level):
    d = cfg["dim"]
    n = 1 << level
    return q_flat.reshape((q_flat.shape[0],) + (n,) * d)


def rk2_step(cfg, q, level, h):
    """One compact RK2 step (Sec. 3) of size h."""
    R1 = rhs(cfg, q, level)
    q1 = q + (h * R1)
    R2 = rhs(cfg, q1, level)
    return ((0.5 * q) + (0.5 * q1)) + ((0.5 * h) * R2)
