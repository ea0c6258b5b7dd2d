"""Remesh pins: brute force on tiny trees, grading invariant, frozen levels.

The paper describes grid adaptation only in words (Alg. AdaptiveMesh,
Alg. waveletThres, "graded tree", "safety" cells, and the LT rule that only
scales evolved in the current iteration may split or merge).  The reading:
significant internal nodes (detail > eps_{l+1}), space safety (existing
neighbours at distance 1), scale safety (children below L), then the least
set closed under the tree rule and the radius-2 grading rule, then the
greatest subset in which every rule still holds with frozen existence at the
lowest changeable level.  The frozen level just below keeps the significance
flags of its last remesh, and their scale safety still seeds its children
(Sec. 4: apart from splitting and merging only between scales at the same
instant, the remesh is the multiresolution one).  This file recomputes that
by naive, randomly ordered fixed-point iteration and compares the oracle's
result.
"""
import itertools

import numpy as np
import pytest

from paper_1905_08717_amd import workloads as W

ABSENT, LEAF, INTERNAL = 0, 1, 2


def _coords(dim, lev, i):
    n = 1 << lev
    return tuple((i // n ** a) % n for a in range(dim))


def _idx(dim, lev, x):
    n = 1 << lev
    return sum(x[a] * n ** a for a in range(dim))


def _nbrs(dim, lev, x, r, periodic):
    n = 1 << lev
    for off in itertools.product(range(-r, r + 1), repeat=dim):
        y = []
        for a in range(dim):
            v = x[a] + off[a]
            if periodic:
                v %= n
            elif v < 0 or v >= n:
                break
            y.append(v)
        else:
            yield tuple(y)


def brute_remesh(dim, L, l0, la, st, D, eps, thresh, periodic, rng, frozen_sig=()):
    """frozen_sig: the significant nodes of level la-1 at its last remesh
    (only those still internal count).  Returns the new statuses and the
    significant nodes of levels la..L-1."""
    eps_l = (lambda lam: eps * 2.0 ** (dim * (lam - L))) if thresh else (lambda lam: eps)
    sig = set()
    for lev in range(la, L):
        for i in np.nonzero(st[lev] == INTERNAL)[0]:
            if eps == 0.0 or D[lev][i] > eps_l(lev + 1):
                sig.add((lev, _coords(dim, lev, int(i))))
    Wset = set(sig)
    for lev, x in sig:
        for y in _nbrs(dim, lev, x, 1, periodic):
            if st[lev][_idx(dim, lev, y)] != ABSENT:
                Wset.add((lev, y))
    scale = set(sig) | {(lev, x) for lev, x in frozen_sig if st[lev][_idx(dim, lev, x)] == INTERNAL}
    for lev, x in scale:
        if lev + 1 <= L - 1:
            for cb in range(1 << dim):
                Wset.add((lev + 1, tuple(2 * x[a] + ((cb >> a) & 1) for a in range(dim))))
    changed = True
    while changed:
        changed = False
        items = list(Wset)
        rng.shuffle(items)
        for lev, x in items:
            if lev <= la:
                continue
            for y in _nbrs(dim, lev, x, 2, periodic):
                p = (lev - 1, tuple(v // 2 for v in y))
                if p not in Wset:
                    Wset.add(p)
                    changed = True

    def exists_new(lev, y):
        if lev == l0:
            return True
        p = tuple(v // 2 for v in y)
        if lev == la:
            return st[lev - 1][_idx(dim, lev - 1, p)] == INTERNAL
        return (lev - 1, p) in Wset

    changed = True
    while changed:
        changed = False
        items = list(Wset)
        rng.shuffle(items)
        for lev, x in items:
            ok = exists_new(lev, x) and all(exists_new(lev, y) for y in _nbrs(dim, lev, x, 2, periodic))
            if not ok:
                Wset.discard((lev, x))
                changed = True
    new = {lev: st[lev].copy() for lev in st}
    for lev in range(la, L + 1):
        for i in range(len(st[lev])):
            x = _coords(dim, lev, i)
            if lev == la:
                if st[lev][i] != ABSENT:
                    new[lev][i] = INTERNAL if (lev, x) in Wset else LEAF
            else:
                p = _idx(dim, lev - 1, tuple(v // 2 for v in x))
                if new[lev - 1][p] == INTERNAL:
                    new[lev][i] = INTERNAL if (lev <= L - 1 and (lev, x) in Wset) else LEAF
                else:
                    new[lev][i] = ABSENT
    return new, sig


def grading_ok(dim, L, l0, st, periodic):
    for lev in range(l0, L):
        for i in np.nonzero(st[lev] == INTERNAL)[0]:
            x = _coords(dim, lev, int(i))
            for y in _nbrs(dim, lev, x, 2, periodic):
                if st[lev][_idx(dim, lev, y)] == ABSENT:
                    return False
            for cb in range(1 << dim):
                y = tuple(2 * x[a] + ((cb >> a) & 1) for a in range(dim))
                if st[lev + 1][_idx(dim, lev + 1, y)] == ABSENT:
                    return False
    return True


CASES = [
    (1, 8, "periodic", 1e-2, 1),
    (1, 8, "neumann", 3e-3, 1),
    (2, 6, "neumann", 2e-2, 1),
    (2, 6, "periodic", 1e-2, 0),
    (3, 4, "neumann", 5e-2, 1),
]


@pytest.mark.parametrize("dim,L,bc,eps,thresh", CASES)
def test_remesh_matches_brute_force_fixed_point(oracle_mod, dim, L, bc, eps, thresh):
    rng = np.random.default_rng(dim * 100 + L)
    l0 = 2
    cfg = dict(dim=dim, L=L, l0=l0, eps=eps, pde="burgers", nu=0.0, bc=bc, thresh=thresh)
    o = oracle_mod.Oracle(cfg)
    n = 1 << L
    # smooth field plus a few sharp features so that several levels appear
    grid = np.meshgrid(*[(np.arange(n) + 0.5) / n] * dim, indexing="ij")
    f = np.sin(2 * np.pi * grid[0])
    for _ in range(3):
        c = rng.uniform(0.2, 0.8, dim)
        r2 = sum((g - cc) ** 2 for g, cc in zip(grid, c))
        f = f + np.where(r2 < rng.uniform(0.005, 0.02), 1.0, 0.0)
    q0 = f.transpose(*reversed(range(dim))).reshape(1, -1)
    o.load_finest(q0)
    periodic = bc == "periodic"
    last_sig = {}   # level -> significant nodes at that level's last remesh
    for la in [l0, l0 + 1, L - 2, L - 1, l0, L - 2, l0 + 1]:
        st = {lev: o.level(lev)[0] for lev in range(l0, L + 1)}
        D = {lev: o.details(lev) for lev in range(l0, L)}
        frozen = last_sig.get(la - 1, set())
        expect, sig = brute_remesh(dim, L, l0, la, st, D, eps, thresh, periodic, rng, frozen)
        for lev in range(la, L):
            last_sig[lev] = {(lv, x) for lv, x in sig if lv == lev}
        o.remesh(la)
        got = {lev: o.level(lev)[0] for lev in range(l0, L + 1)}
        for lev in range(l0, L + 1):
            assert np.array_equal(got[lev], expect[lev]), (la, lev)
            if lev <= la:
                assert np.array_equal(got[lev] != ABSENT, st[lev] != ABSENT), (la, lev)
            if lev < la:
                assert np.array_equal(got[lev], st[lev])
        assert grading_ok(dim, L, l0, got, periodic)
        assert len({int(v) for lev in range(l0, L + 1) for v in np.unique(got[lev])}) >= 2


def test_remesh_values_of_new_and_merged_nodes(oracle_mod):
    # merged parents keep the projection of their children (Sec. 2); new
    # children are predicted from the parent level, so projection of the new
    # children returns the parent value (consistency of the prediction).
    cfg = W.burgers_1d(L=8, eps=1e-2)
    o = oracle_mod.Oracle(cfg)
    q = W.burgers_sine(8)
    q[0, 100:110] += 1.0
    o.load_finest(q)
    keys0, v0 = o.get_leaves()
    total0 = (v0[0] / 2.0 ** (keys0 >> np.uint64(56)).astype(float)).sum()
    o.remesh(2)
    keys1, v1 = o.get_leaves()
    total1 = (v1[0] / 2.0 ** (keys1 >> np.uint64(56)).astype(float)).sum()
    assert abs(total1 - total0) < 1e-13


def test_adapt_keeps_all_with_eps_zero(oracle_mod):
    cfg = W.nagumo_2d(L=5, eps=0.0)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(W.nagumo_front(5))
    st = o.stats()
    assert st["leaves"][5] == 1024 and sum(st["leaves"]) == 1024


@pytest.mark.parametrize("case", ["nagumo2d", "flameball3d", "euler2d"])
def test_remesh_of_synchronised_data_keeps_the_adapted_tree(oracle_mod, case):
    """Without time evolution, a remesh with levels below la frozen must give
    the tree that the full remesh gave (Sec. 4: apart from which scales may
    split or merge, the LT remesh is the multiresolution remesh).  Dropping
    the frozen level's scale safety would merge every node that only its
    significant parent kept refined."""
    if case == "nagumo2d":
        cfg, q0 = W.nagumo_2d(L=7), W.nagumo_front(7)
    elif case == "flameball3d":
        cfg, q0 = W.flame_ball_3d(L=5), W.flame_ball(5)
    else:
        cfg, q0 = W.euler_2d(L=6), W.euler_quadrants_seeded(6, W.SEED)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(q0)
    L, l0 = cfg["L"], cfg["l0"]
    ref = {lev: o.level(lev)[0].copy() for lev in range(l0, L + 1)}
    for la in list(range(l0 + 1, L)) + [l0]:
        o.remesh(la)
        for lev in range(l0, L + 1):
            assert np.array_equal(o.level(lev)[0], ref[lev]), (la, lev)


def test_near_threshold_decision_is_recorded(oracle_mod):
    """A threshold equal to a computed detail (Alg. waveletThres keeps a
    node only when its detail exceeds the threshold): the node is not
    significant, and the decision is listed as near the threshold with the
    iteration, level and Morton key of the node."""
    from tests.trees import morton_encode
    cfg = W.nagumo_2d(L=6, eps=0.0)
    q0 = W.nagumo_front(6)
    o = oracle_mod.Oracle(cfg)
    o.load_finest(q0)
    assert o.near_threshold() == []          # eps = 0: no threshold test
    D = o.details(4)                          # level-4 nodes, details of level-5 children
    i = int(np.argsort(D)[-40])               # a node well inside the front
    assert D[i] > 0
    eps = D[i] * 4.0                          # eps_5 = 2^{2 (5 - 6)} eps = D exactly
    o2 = oracle_mod.Oracle(dict(cfg, eps=eps))
    o2.load_finest(q0)
    key = morton_encode(2, (i % 16, i // 16))
    near = o2.near_threshold()
    assert (0, 4, key) in near
    assert o2.stats()["near_threshold"] == len(near)
