"""List codes of 16-cell Morton groups (the compaction's classification):
the bit-parallel form in group_codes.h against a cell-by-cell reading of
the definitions, on random status neighbourhoods in 1D, 2D and 3D.

Leaf: every leaf; internal: every internal node; interface leaf: a leaf
with an internal cell at offset +-1 (and +-2 when the stencil reaches two
cells) along an axis; virtual cell: an absent cell whose parent is a leaf
and that has a leaf at offset +-1 or +-2 along an axis (Fig. 1, Sec. 2);
in 1D and 2D, bit 16 << (2a + s) of a leaf: its face neighbour along axis
a (s = 0 below, 1 above) is absent, the fine side of a refined face (no
list).  Cells outside the domain count as none of these."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1905_08717_amd", "csrc")

WIDTH = {1: (16, 1, 1), 2: (4, 4, 1), 3: (4, 2, 2)}


def morton(D, x, y, z):
    """Morton index of a cell of the group from its local coordinates."""
    if D == 1:
        return x
    if D == 2:
        return (x & 1) | ((y & 1) << 1) | ((x >> 1) << 2) | ((y >> 1) << 3)
    return (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((x >> 1) << 3)


def reference(D, reach, c, m, p, par):
    """codes per Morton cell from the statuses (lists of 16 ints; m[a] /
    p[a] None outside the domain)."""
    w = WIDTH[D]
    codes = [0] * 16
    for z in range(w[2]):
        for y in range(w[1]):
            for x in range(w[0]):
                j = morton(D, x, y, z)
                st = c[j]

                def nb(a, o):
                    u = [x, y, z]
                    u[a] += o
                    if 0 <= u[a] < w[a]:
                        return c[morton(D, *u)]
                    grp = p[a] if u[a] >= w[a] else m[a]
                    if grp is None:
                        return 3
                    u[a] %= w[a]
                    return grp[morton(D, *u)]

                if st == 2:
                    codes[j] = 2
                elif st == 1:
                    offs = (-2, -1, 1, 2) if reach == 2 else (-1, 1)
                    iface = any(nb(a, o) == 2 for a in range(D) for o in offs)
                    faces = 0
                    if D <= 2:
                        for a in range(D):
                            for sd, o in enumerate((-1, 1)):
                                if nb(a, o) == 0:
                                    faces |= 16 << (2 * a + sd)
                    codes[j] = 1 | (4 if iface else 0) | faces
                else:
                    pleaf = par[j >> D] == 1
                    near = any(nb(a, o) == 1 for a in range(D) for o in (-2, -1, 1, 2))
                    codes[j] = 8 if (pleaf and near) else 0
    return codes


def words(b):
    return [int(b[4 * q]) | (int(b[4 * q + 1]) << 8) | (int(b[4 * q + 2]) << 16) | (int(b[4 * q + 3]) << 24)
            for q in range(4)]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("gc") / "gc")
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-I", CSRC, os.path.join(HERE, "native", "group_codes_driver.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("D", [1, 2, 3])
def test_bit_parallel_codes_match_the_definitions(driver, D):
    rng = np.random.default_rng(7 + D)
    cases, refs = [], []
    for i in range(3000):
        # mixtures from all-internal to sparse leaves, so every code occurs
        pr = rng.dirichlet([1.0, 1.0, 1.0])
        draw = lambda: list(rng.choice(3, size=16, p=pr))
        reach = 1 + (i % 2)
        c = draw()
        m = [None if rng.random() < 0.15 else draw() for _ in range(D)]
        p = [None if rng.random() < 0.15 else draw() for _ in range(D)]
        par = list(rng.choice(3, size=16 >> D, p=[0.2, 0.5, 0.3]))
        line = [str(D), str(reach)] + ["%x" % v for v in words(c)]
        for a in range(D):
            line += ["%x" % v for v in words(m[a] or [0] * 16)]
        for a in range(D):
            line += ["%x" % v for v in words(p[a] or [0] * 16)]
        outside = sum((1 << (2 * a)) * (m[a] is None) + (1 << (2 * a + 1)) * (p[a] is None) for a in range(D))
        line.append("%x" % outside)
        line.append("%x" % sum(int(s) << (8 * k) for k, s in enumerate(par)))
        cases.append(" ".join(line))
        refs.append(reference(D, reach, c, m, p, par))
    out = subprocess.run([driver], input="\n".join(cases) + "\n", capture_output=True, text=True, check=True)
    lines = out.stdout.split("\n")
    seen = set()
    for ref, ln in zip(refs, lines):
        f = ln.split()
        got = []
        for q in range(4):
            v = int(f[q], 16)
            got += [(v >> (8 * b)) & 0xFF for b in range(4)]
        assert got == ref
        cnt = int(f[4], 16)
        want = [sum(1 for r in ref if r & bit) for bit in (1, 2, 4, 8)]
        assert [(cnt >> (16 * k)) & 0xFFFF for k in range(4)] == want
        seen.update(ref)
    assert {0, 1, 2, 5, 8} <= seen
    if D <= 2:  # every face bit occurs, with and without the interface bit
        assert all(any(r & (16 << f) for r in seen) for f in range(2 * D))
        assert any(r & 4 and r & 0xF0 for r in seen)
