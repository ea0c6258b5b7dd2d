"""ctypes wrapper of the CPU oracle (``oracle/mro.c``).

TEST INFRASTRUCTURE ONLY: the oracle is a plain FP64 CPU implementation of
the MRLT/NERK3 macro step of arXiv:1905.08717, used to check the HIP path.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the package
``paper_1905_08717_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmro.so")
SRC = os.path.join(HERE, "mro.c")

PDE = {"advection": 0, "burgers": 1, "nagumo": 2, "euler": 3, "linear": 4, "flame": 5, "flameball": 6}
BC = {"periodic": 0, "neumann": 1, "dirichlet": 2}

OK, EINVAL, ENOMEM, ESTATE, ENONFINITE = 0, -1, -2, -4, -5
MAXLEV = 30


class Scheme(ctypes.Structure):
    _fields_ = [
        ("pde", ctypes.c_int32), ("rk", ctypes.c_int32), ("lt", ctypes.c_int32),
        ("l0", ctypes.c_int32), ("recon", ctypes.c_int32), ("thresh", ctypes.c_int32),
        ("reflux", ctypes.c_int32), ("remesh", ctypes.c_int32),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("nu", ctypes.c_double), ("k_react", ctypes.c_double), ("a_react", ctypes.c_double),
        ("gamma", ctypes.c_double), ("adv_vel", ctypes.c_double * 3),
        ("detail_scale", ctypes.c_double * 5),
        ("ze", ctypes.c_double), ("tau", ctypes.c_double), ("lewis", ctypes.c_double),
        ("kappa", ctypes.c_double), ("flame_speed", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("leaves", ctypes.c_int64 * (MAXLEV + 1)),
        ("leaf_updates", ctypes.c_int64),
        ("near_threshold", ctypes.c_int64),
        ("iterations", ctypes.c_int64),
        ("mass", ctypes.c_double * 5),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "mro.h"))
    ):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.mro_init.argtypes = [i32, i32, dbl, ctypes.POINTER(Scheme), ctypes.POINTER(vp)]
        L.mro_destroy.argtypes = [vp]
        L.mro_destroy.restype = None
        L.mro_ncomp.argtypes = [vp]
        L.mro_num_threads.argtypes = []
        L.mro_load_finest.argtypes = [vp, dp]
        L.mro_adapt.argtypes = [vp]
        L.mro_lt_step.argtypes = [vp, dbl]
        L.mro_reconstruct.argtypes = [vp, dp]
        L.mro_max_wavespeed.argtypes = [vp, dp]
        L.mro_flame_speed.argtypes = [vp, dp]
        L.mro_get_leaves.argtypes = [vp, u64p, dp, i64, ctypes.POINTER(i64)]
        L.mro_set_leaves.argtypes = [vp, u64p, dp, i64, dbl]
        L.mro_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.mro_last_error.argtypes = [vp]
        L.mro_last_error.restype = ctypes.c_char_p
        L.mro_get_level.argtypes = [vp, i32, u8p, dp]
        L.mro_remesh.argtypes = [vp, i32]
        L.mro_predict.argtypes = [i32, i32, dp, dp]
        L.mro_project.argtypes = [i32, i32, dp, dp]
        L.mro_face_flux.argtypes = [vp, i32, i32, dp, dp]
        L.mro_details.argtypes = [vp, i32, dp]
        L.mro_near_threshold.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32), u64p, i64,
                                         ctypes.POINTER(i64)]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_scheme(cfg: dict) -> Scheme:
    """Fill the oracle's scheme struct from a plain configuration dict."""
    s = Scheme()
    d = cfg["dim"]
    s.pde = PDE[cfg["pde"]]
    s.rk = cfg.get("rk", 3)
    s.lt = cfg.get("lt", 1)
    s.l0 = cfg.get("l0", 2)
    s.recon = cfg.get("recon", 1)
    s.thresh = cfg.get("thresh", 1)
    s.reflux = cfg.get("reflux", 1)
    s.remesh = cfg.get("remesh", 1)
    bc = cfg.get("bc", "periodic")
    for a in range(3):
        b = bc[a] if isinstance(bc, (list, tuple)) else bc
        lo_hi = b if isinstance(b, (list, tuple)) else (b, b)   # per side or both
        s.bc[a][0] = BC[lo_hi[0]]
        s.bc[a][1] = BC[lo_hi[1]]
        s.lo[a] = cfg.get("lo", [0.0] * 3)[a] if a < d else 0.0
        s.hi[a] = cfg.get("hi", [1.0] * 3)[a] if a < d else 1.0
    s.nu = cfg.get("nu", 0.0)
    s.k_react = cfg.get("k_react", 0.0)
    s.a_react = cfg.get("a_react", 0.0)
    s.gamma = cfg.get("gamma", 1.4)
    v = cfg.get("adv_vel", [1.0, 0.0, 0.0])
    for a in range(3):
        s.adv_vel[a] = v[a]
    sc = cfg.get("detail_scale", [1.0] * 5)
    for k in range(5):
        s.detail_scale[k] = sc[k]
    s.ze = cfg.get("ze", 0.0)
    s.tau = cfg.get("tau", 0.0)
    s.lewis = cfg.get("lewis", 1.0)
    s.kappa = cfg.get("kappa", 0.0)
    s.flame_speed = cfg.get("flame_speed", 0)
    return s


class OracleError(RuntimeError):
    pass


class Oracle:
    """One solve held by the CPU oracle."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.dim, self.L = cfg["dim"], cfg["L"]
        self.l0 = cfg.get("l0", 2)
        self._s = make_scheme(cfg)
        h = ctypes.c_void_p()
        rc = lib().mro_init(self.dim, self.L, float(cfg["eps"]), ctypes.byref(self._s), ctypes.byref(h))
        if rc != OK:
            raise OracleError(f"mro_init failed ({rc})")
        self._h = h
        self.m = lib().mro_ncomp(h)
        self.nfine = 1 << (self.dim * self.L)

    def close(self):
        if getattr(self, "_h", None):
            lib().mro_destroy(self._h)
            self._h = None

    __del__ = close

    def _check(self, rc, what):
        if rc != OK:
            msg = lib().mro_last_error(self._h)
            raise OracleError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def load_finest(self, q0: np.ndarray):
        q = np.ascontiguousarray(q0, dtype=np.float64).reshape(self.m, self.nfine)
        self._check(lib().mro_load_finest(self._h, _dp(q)), "mro_load_finest")

    def adapt(self):
        self._check(lib().mro_adapt(self._h), "mro_adapt")

    def lt_step(self, dt: float):
        rc = lib().mro_lt_step(self._h, float(dt))
        self._check(rc, "mro_lt_step")

    def lt_step_rc(self, dt: float) -> int:
        return lib().mro_lt_step(self._h, float(dt))

    def reconstruct(self) -> np.ndarray:
        out = np.zeros((self.m, self.nfine))
        self._check(lib().mro_reconstruct(self._h, _dp(out)), "mro_reconstruct")
        return out

    def max_wavespeed(self) -> float:
        v = ctypes.c_double()
        self._check(lib().mro_max_wavespeed(self._h, ctypes.byref(v)), "mro_max_wavespeed")
        return v.value

    def flame_speed(self) -> float:
        """v_f of the current leaves: the reaction rate integrated over the
        domain per unit cross-section (Sec. 5)."""
        v = ctypes.c_double()
        self._check(lib().mro_flame_speed(self._h, ctypes.byref(v)), "mro_flame_speed")
        return v.value

    def get_leaves(self):
        n = ctypes.c_int64()
        self._check(lib().mro_get_leaves(self._h, None, None, 0, ctypes.byref(n)), "mro_get_leaves")
        keys = np.zeros(n.value, dtype=np.uint64)
        q = np.zeros((self.m, n.value))
        self._check(
            lib().mro_get_leaves(self._h, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dp(q),
                                 n.value, ctypes.byref(n)), "mro_get_leaves")
        return keys, q

    def set_leaves(self, keys: np.ndarray, q: np.ndarray, t: float = 0.0):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(self.m, len(keys))
        self._check(
            lib().mro_set_leaves(self._h, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dp(q),
                                 len(keys), float(t)), "mro_set_leaves")

    def stats(self) -> dict:
        st = Stats()
        self._check(lib().mro_stats(self._h, ctypes.byref(st)), "mro_stats")
        return {
            "t": st.t,
            "leaves": [st.leaves[i] for i in range(MAXLEV + 1)],
            "leaf_updates": st.leaf_updates,
            "near_threshold": st.near_threshold,
            "iterations": st.iterations,
            "mass": [st.mass[k] for k in range(self.m)],
        }

    def near_threshold(self):
        """Near-threshold decisions since the last load / set_leaves as a
        sorted list of (iteration, level, Morton key)."""
        n = ctypes.c_int64()
        self._check(lib().mro_near_threshold(self._h, None, None, None, 0, ctypes.byref(n)), "mro_near_threshold")
        it = np.zeros(n.value, dtype=np.int64)
        lv = np.zeros(n.value, dtype=np.int32)
        ky = np.zeros(n.value, dtype=np.uint64)
        if n.value:
            self._check(lib().mro_near_threshold(
                self._h, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                ky.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n.value, ctypes.byref(n)), "mro_near_threshold")
        return [(int(a), int(b), int(c)) for a, b, c in zip(it, lv, ky)]

    def level(self, lev: int):
        n = 1 << (self.dim * lev)
        status = np.zeros(n, dtype=np.uint8)
        q0 = np.zeros((self.m, n))
        self._check(lib().mro_get_level(self._h, lev, status.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        _dp(q0)), "mro_get_level")
        return status, q0

    def remesh(self, la: int):
        self._check(lib().mro_remesh(self._h, la), "mro_remesh")

    def details(self, lev: int) -> np.ndarray:
        D = np.zeros(1 << (self.dim * lev))
        self._check(lib().mro_details(self._h, lev, _dp(D)), "mro_details")
        return D

    def face_flux(self, lev: int, direction: int, cells: np.ndarray) -> np.ndarray:
        c = np.ascontiguousarray(cells, dtype=np.float64).reshape(4, self.m)
        F = np.zeros(self.m)
        self._check(lib().mro_face_flux(self._h, lev, direction, _dp(c), _dp(F)), "mro_face_flux")
        return F


def num_threads() -> int:
    return lib().mro_num_threads()


def predict(dim: int, stencil: np.ndarray) -> np.ndarray:
    """Children (2^d, m) predicted from a (m, 27) stencil."""
    st = np.ascontiguousarray(stencil, dtype=np.float64).reshape(-1, 27)
    m = st.shape[0]
    out = np.zeros((1 << dim, m))
    rc = lib().mro_predict(dim, m, _dp(st), _dp(out))
    assert rc == OK
    return out


def project(dim: int, children: np.ndarray) -> np.ndarray:
    ch = np.ascontiguousarray(children, dtype=np.float64).reshape(1 << dim, -1)
    m = ch.shape[1]
    out = np.zeros(m)
    rc = lib().mro_project(dim, m, _dp(ch), _dp(out))
    assert rc == OK
    return out


def morton_decode(dim: int, key: int):
    x = [0, 0, 0]
    for b in range(21):
        for a in range(dim):
            x[a] |= ((key >> (dim * b + a)) & 1) << b
    return x[:dim]


def morton_encode(dim: int, x) -> int:
    k = 0
    for b in range(21):
        for a in range(dim):
            k |= ((int(x[a]) >> b) & 1) << (dim * b + a)
    return k


def leaf_key(level: int, dim: int, x) -> int:
    return (level << 56) | morton_encode(dim, x)
