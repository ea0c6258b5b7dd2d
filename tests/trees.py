"""Helpers that build graded trees and leaf values for tests."""
from __future__ import annotations

import itertools

import numpy as np

from paper_1905_08717_amd.workloads import SEED  # noqa: F401  (re-export for tests)


def morton_encode(dim: int, x) -> int:
    k = 0
    for b in range(21):
        for a in range(dim):
            k |= ((int(x[a]) >> b) & 1) << (dim * b + a)
    return k


def leaf_key(level: int, dim: int, x) -> int:
    return (level << 56) | morton_encode(dim, x)


def build_tree(dim: int, L: int, l0: int, levfn):
    """Leaves (level, coords) of the tree that refines every cell whose
    centre asks for a finer level (levfn(centre) > level), from level l0."""
    leaves = []

    def rec(lev, x):
        centre = [(x[a] + 0.5) / (1 << lev) for a in range(dim)]
        if lev < L and levfn(centre) > lev:
            for cb in range(1 << dim):
                rec(lev + 1, [2 * x[a] + ((cb >> a) & 1) for a in range(dim)])
        else:
            leaves.append((lev, tuple(x)))

    for idx in itertools.product(range(1 << l0), repeat=dim):
        rec(l0, list(idx))
    leaves.sort(key=lambda lx: leaf_key(lx[0], dim, lx[1]))
    return leaves


def leaf_arrays(dim: int, leaves, valfn, m: int = 1):
    """Keys sorted by (level, Morton) and values (m, n) from valfn(level, x)."""
    keys = np.array([leaf_key(lev, dim, x) for lev, x in leaves], dtype=np.uint64)
    vals = np.zeros((m, len(leaves)))
    for j, (lev, x) in enumerate(leaves):
        vals[:, j] = valfn(lev, x)
    return keys, vals


def box_average_poly(dim: int, lev: int, x, coeffs, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Exact average over cell x at level lev of sum_a c_a * x_a^2 (coeffs c_a)."""
    tot = 0.0
    for a in range(dim):
        h = (hi[a] - lo[a]) / (1 << lev)
        l = lo[a] + x[a] * h
        r = l + h
        tot += coeffs[a] * (r ** 3 - l ** 3) / (3.0 * h)
    return tot
