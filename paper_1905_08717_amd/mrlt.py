"""Thin Python binding of libmrlt.so (the C ABI in include/mrlt.h).

Argument marshalling only: every step of the macro step runs in the HIP
library.  Device buffers are torch tensors on a HIP device (PyTorch is used
for device memory and streams).  Loading fails loudly when the library has
not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrlt.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE, ECAPACITY = 0, -1, -2, -3, -4, -5, -6
PDE = {"advection": 0, "burgers": 1, "nagumo": 2, "euler": 3, "linear": 4, "flame": 5, "flameball": 6}
BC = {"periodic": 0, "neumann": 1, "dirichlet": 2}
MAXLEV = 24

# every symbol declared in include/mrlt.h
EXPORTS = [
    "mr_init", "mr_init_batch", "mr_set_stream", "mr_ncomp", "mr_load_finest", "mr_adapt",
    "mr_lt_step", "mr_lt_step_batch", "mr_reconstruct", "mr_max_wavespeed", "mr_get_leaves",
    "mr_get_leaves_inst", "mr_set_leaves", "mr_set_leaves_inst", "mr_stats", "mr_stats_inst",
    "mr_synchronize", "mr_last_error", "mr_destroy", "mr_level_updates", "mr_timing_start",
    "mr_timing_stop", "mr_load_finest_inst", "mr_clear_instance", "mr_instance_flags", "mr_set_eps",
    "mr_stage_items", "mr_flame_speed", "mr_set_launch", "mr_get_launch", "mr_near_threshold",
    "mr_get_leaves_noalloc", "mr_load_inst", "mr_footprint",
    "mr_batch_create", "mr_batch_admit", "mr_batch_step", "mr_batch_poll", "mr_batch_slot_info",
    "mr_batch_get_leaves", "mr_batch_release", "mr_batch_footprint", "mr_batch_last_error", "mr_batch_destroy",
]
SLOT_FREE, SLOT_RUNNING, SLOT_DONE, SLOT_FAILED = 0, 1, 2, 3
KC = {"stage_finest": 1, "stage": 2, "project": 3, "ghost": 4, "remesh": 5, "finalize": 6, "stage_bulk": 7}


class MrScheme(ctypes.Structure):
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


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class MrAlloc(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class MrClassDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("L_max", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("scheme", MrScheme)]


class MrInstanceDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("eps", ctypes.c_double),
                ("t_final", ctypes.c_double), ("cfl", ctypes.c_double), ("dt_max", ctypes.c_double),
                ("scheme", MrScheme)]


class MrLaunch(ctypes.Structure):
    _fields_ = [("list_grid", ctypes.c_int32), ("iface_grid", ctypes.c_int32), ("comp_grid", ctypes.c_int32),
                ("bulk_levels", ctypes.c_int32)]


class MrStats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("leaves", ctypes.c_int64 * (MAXLEV + 1)),
        ("leaf_updates", ctypes.c_int64),
        ("near_threshold", ctypes.c_int64),
        ("iterations", ctypes.c_int64),
        ("mass", ctypes.c_double * 5),
    ]


class MrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load_library():
    """Load libmrlt.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1905_08717_amd/build.py "
                          "(the HIP path has no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    sp = ctypes.POINTER(MrScheme)
    ap = ctypes.POINTER(MrAlloc)
    L.mr_init.argtypes = [i32, i32, dbl, sp, ap, ctypes.POINTER(vp)]
    L.mr_init_batch.argtypes = [i32, i32, i32, dp, sp, ap, ctypes.POINTER(vp)]
    L.mr_footprint.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mr_batch_create.argtypes = [i32, ctypes.POINTER(MrClassDesc), ctypes.c_size_t, ap, ctypes.POINTER(vp)]
    L.mr_batch_admit.argtypes = [vp, ctypes.POINTER(MrInstanceDesc), vp, ctypes.POINTER(i32)]
    L.mr_batch_step.argtypes = [vp]
    L.mr_batch_poll.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
    L.mr_batch_slot_info.argtypes = [vp, i32, ctypes.POINTER(i32), dp, ctypes.POINTER(i64)]
    L.mr_batch_get_leaves.argtypes = [vp, i32, u64p, dp, i64, ctypes.POINTER(i64)]
    L.mr_batch_release.argtypes = [vp, i32]
    L.mr_batch_footprint.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mr_batch_last_error.argtypes = [vp]
    L.mr_batch_last_error.restype = ctypes.c_char_p
    L.mr_batch_destroy.argtypes = [vp]
    L.mr_batch_destroy.restype = None
    L.mr_set_stream.argtypes = [vp, vp]
    L.mr_ncomp.argtypes = [vp]
    L.mr_load_finest.argtypes = [vp, vp, vp]
    L.mr_adapt.argtypes = [vp]
    L.mr_lt_step.argtypes = [vp, dbl]
    L.mr_lt_step_batch.argtypes = [vp, dp]
    L.mr_reconstruct.argtypes = [vp, vp]
    L.mr_max_wavespeed.argtypes = [vp, dp]
    L.mr_flame_speed.argtypes = [vp, dp]
    L.mr_set_launch.argtypes = [vp, ctypes.POINTER(MrLaunch)]
    L.mr_get_launch.argtypes = [vp, ctypes.POINTER(MrLaunch)]
    L.mr_get_leaves.argtypes = [vp, u64p, dp, i64, ctypes.POINTER(i64)]
    L.mr_get_leaves_inst.argtypes = [vp, i32, u64p, dp, i64, ctypes.POINTER(i64)]
    L.mr_get_leaves_noalloc.argtypes = [vp, i32, u64p, dp, i64, ctypes.POINTER(i64)]
    L.mr_set_leaves.argtypes = [vp, u64p, dp, i64, dbl]
    L.mr_set_leaves_inst.argtypes = [vp, i32, u64p, dp, i64, dbl]
    L.mr_stats.argtypes = [vp, ctypes.POINTER(MrStats)]
    L.mr_stats_inst.argtypes = [vp, i32, ctypes.POINTER(MrStats)]
    L.mr_synchronize.argtypes = [vp]
    L.mr_last_error.argtypes = [vp]
    L.mr_last_error.restype = ctypes.c_char_p
    L.mr_level_updates.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.mr_timing_start.argtypes = [vp, i32]
    L.mr_stage_items.argtypes = [vp, ctypes.POINTER(i64)]
    L.mr_timing_stop.argtypes = [vp, dp, ctypes.POINTER(i64)]
    L.mr_load_finest_inst.argtypes = [vp, i32, vp]
    L.mr_load_inst.argtypes = [vp, i32, i32, dbl, vp]
    L.mr_clear_instance.argtypes = [vp, i32]
    L.mr_instance_flags.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.mr_set_eps.argtypes = [vp, i32, dbl]
    L.mr_near_threshold.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32), u64p, i64,
                                    ctypes.POINTER(i64)]
    L.mr_destroy.argtypes = [vp]
    L.mr_destroy.restype = None
    for name in EXPORTS:
        if name not in ("mr_last_error", "mr_destroy", "mr_ncomp", "mr_batch_last_error", "mr_batch_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def make_scheme(cfg: dict) -> MrScheme:
    s = MrScheme()
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


_TORCH_ALLOC = None


def torch_allocator() -> MrAlloc:
    """Device memory from PyTorch's caching allocator (the mr_alloc
    callbacks of the C ABI); the callback objects live for the process."""
    global _TORCH_ALLOC
    if _TORCH_ALLOC is None:
        import torch

        def _alloc(nbytes, _user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:   # out of memory: the library reports MR_ENOMEM
                return None

        def _free(ptr, _user):
            torch.cuda.caching_allocator_delete(int(ptr))

        _TORCH_ALLOC = MrAlloc(ALLOC_FN(_alloc), FREE_FN(_free), None)
    return _TORCH_ALLOC


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(int(stream.cuda_stream))


class Solver:
    """A batch of MRLT/NERK3 solves on one GPU (n_inst = 1 for a single solve)."""

    def __init__(self, cfg: dict, n_inst: int = 1, eps=None, stream=None, alloc: MrAlloc = None):
        import torch

        self.torch = torch
        L = load_library()
        self.cfg = dict(cfg)
        self.dim, self.L = cfg["dim"], cfg["L"]
        self.n_inst = n_inst
        if eps is None:
            eps = [cfg["eps"]] * n_inst
        eps_arr = (ctypes.c_double * n_inst)(*[float(e) for e in eps])
        self._s = make_scheme(cfg)
        h = ctypes.c_void_p()
        self._h = None
        self._alloc = alloc
        rc = L.mr_init_batch(self.dim, self.L, n_inst, eps_arr, ctypes.byref(self._s),
                             ctypes.byref(alloc) if alloc is not None else None, ctypes.byref(h))
        if rc != OK:
            raise MrError(rc, "mr_init_batch failed")
        self._h = h
        self.m = L.mr_ncomp(h)
        self.nfine = 1 << (self.dim * self.L)
        # the library queues on its own stream unless one is given; device
        # buffers written by torch are synchronised before they are read
        self.stream = stream
        self._check(L.mr_set_stream(h, _stream_ptr(stream)), "mr_set_stream")

    def close(self):
        if getattr(self, "_h", None):
            load_library().mr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            msg = load_library().mr_last_error(self._h) if self._h else b""
            raise MrError(rc, f"{what} failed: {msg.decode() if msg else ''}")

    def load_finest(self, q0):
        """q0: torch FP64 device tensor [n_inst, m, 2^{dL}] (or numpy, copied)."""
        t = self.torch
        if isinstance(q0, np.ndarray):
            q0 = t.from_numpy(np.ascontiguousarray(q0, dtype=np.float64)).to("cuda")
        q0 = q0.contiguous()
        assert q0.dtype == t.float64 and q0.is_cuda and q0.numel() == self.n_inst * self.m * self.nfine
        t.cuda.current_stream().synchronize()
        self._q0_keep = q0
        self._check(load_library().mr_load_finest(self._h, ctypes.c_void_p(q0.data_ptr()),
                                                  _stream_ptr(self.stream)), "mr_load_finest")

    def load_finest_inst(self, inst: int, q0):
        """Load one instance (q0: [m, 2^{dL}], torch device tensor or numpy)."""
        t = self.torch
        if isinstance(q0, np.ndarray):
            q0 = t.from_numpy(np.ascontiguousarray(q0, dtype=np.float64)).to("cuda")
        q0 = q0.contiguous()
        assert q0.dtype == t.float64 and q0.is_cuda and q0.numel() == self.m * self.nfine
        t.cuda.current_stream().synchronize()
        self._keep_inst = q0
        self._check(load_library().mr_load_finest_inst(self._h, inst, ctypes.c_void_p(q0.data_ptr())),
                    "mr_load_finest_inst")

    def load_inst(self, inst: int, L_inst: int, eps: float, q0):
        """Load one instance with its own finest level L_inst <= L and
        threshold eps (q0: [m, 2^{d L_inst}], torch device tensor or numpy);
        step it with dt_L = 2^{L_inst - L} times its own finest step."""
        t = self.torch
        if isinstance(q0, np.ndarray):
            q0 = t.from_numpy(np.ascontiguousarray(q0, dtype=np.float64)).to("cuda")
        q0 = q0.contiguous()
        assert q0.dtype == t.float64 and q0.is_cuda and q0.numel() == self.m * (1 << (self.dim * L_inst))
        t.cuda.current_stream().synchronize()
        self._keep_inst = q0
        self._check(load_library().mr_load_inst(self._h, inst, int(L_inst), float(eps),
                                                ctypes.c_void_p(q0.data_ptr())), "mr_load_inst")

    def clear_instance(self, inst: int):
        self._check(load_library().mr_clear_instance(self._h, inst), "mr_clear_instance")

    def instance_flags(self, inst: int) -> int:
        f = ctypes.c_int()
        self._check(load_library().mr_instance_flags(self._h, inst, ctypes.byref(f)), "mr_instance_flags")
        return f.value

    def set_eps(self, inst: int, eps: float):
        self._check(load_library().mr_set_eps(self._h, inst, float(eps)), "mr_set_eps")

    def last_error(self) -> str:
        msg = load_library().mr_last_error(self._h)
        return msg.decode() if msg else ""

    def lt_step_rc_batch(self, dts) -> int:
        arr = (ctypes.c_double * self.n_inst)(*[float(x) for x in dts])
        return load_library().mr_lt_step_batch(self._h, arr)

    def adapt(self):
        self._check(load_library().mr_adapt(self._h), "mr_adapt")

    def lt_step(self, dt):
        if np.ndim(dt) == 0:
            self._check(load_library().mr_lt_step(self._h, float(dt)), "mr_lt_step")
        else:
            arr = (ctypes.c_double * self.n_inst)(*[float(x) for x in dt])
            self._check(load_library().mr_lt_step_batch(self._h, arr), "mr_lt_step_batch")

    def lt_step_rc(self, dt) -> int:
        return load_library().mr_lt_step(self._h, float(dt))

    def reconstruct(self):
        out = self.torch.empty((self.n_inst, self.m, self.nfine), dtype=self.torch.float64, device="cuda")
        self.torch.cuda.current_stream().synchronize()
        self._check(load_library().mr_reconstruct(self._h, ctypes.c_void_p(out.data_ptr())), "mr_reconstruct")
        return out

    def max_wavespeed(self):
        arr = (ctypes.c_double * self.n_inst)()
        self._check(load_library().mr_max_wavespeed(self._h, arr), "mr_max_wavespeed")
        return np.array(arr[:])

    def set_launch(self, list_grid: int = 0, iface_grid: int = 0, comp_grid: int = 0, bulk_levels: int = 0):
        """Grid caps of the list-driven kernels, the interface-leaf stage
        launches and the compaction, and the bulk stage kernel's
        block-to-level schedule (1: one launch over all levels of a stage,
        2: one per level); 0 keeps a value; results do not depend on them."""
        lc = MrLaunch(int(list_grid), int(iface_grid), int(comp_grid), int(bulk_levels))
        self._check(load_library().mr_set_launch(self._h, ctypes.byref(lc)), "mr_set_launch")

    def get_launch(self) -> dict:
        lc = MrLaunch()
        self._check(load_library().mr_get_launch(self._h, ctypes.byref(lc)), "mr_get_launch")
        return {"list_grid": lc.list_grid, "iface_grid": lc.iface_grid, "comp_grid": lc.comp_grid,
                "bulk_levels": lc.bulk_levels}

    def flame_speed(self):
        """v_f of every instance from its current leaves (flame problems)."""
        arr = (ctypes.c_double * self.n_inst)()
        self._check(load_library().mr_flame_speed(self._h, arr), "mr_flame_speed")
        return np.array(arr[:])

    def get_leaves(self, inst: int = 0):
        L = load_library()
        n = ctypes.c_int64()
        self._check(L.mr_get_leaves_inst(self._h, inst, None, None, 0, ctypes.byref(n)), "mr_get_leaves")
        keys = np.zeros(n.value, dtype=np.uint64)
        q = np.zeros((self.m, n.value))
        self._check(L.mr_get_leaves_inst(self._h, inst, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                         q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
                                         ctypes.byref(n)), "mr_get_leaves")
        return keys, q

    def get_leaves_noalloc(self, inst: int = 0):
        """Leaves of one instance through the library's fixed staging array
        (mr_get_leaves_noalloc): no device allocation in the call."""
        L = load_library()
        n = ctypes.c_int64()
        self._check(L.mr_get_leaves_noalloc(self._h, inst, None, None, 0, ctypes.byref(n)), "mr_get_leaves_noalloc")
        keys = np.zeros(n.value, dtype=np.uint64)
        q = np.zeros((self.m, n.value))
        self._check(L.mr_get_leaves_noalloc(self._h, inst, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                            q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
                                            ctypes.byref(n)), "mr_get_leaves_noalloc")
        return keys, q

    def set_leaves(self, keys, q, t: float = 0.0, inst: int = 0):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(self.m, len(keys))
        self._check(load_library().mr_set_leaves_inst(
            self._h, inst, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(keys), float(t)), "mr_set_leaves")

    def stats(self, inst: int = 0) -> dict:
        st = MrStats()
        self._check(load_library().mr_stats_inst(self._h, inst, ctypes.byref(st)), "mr_stats")
        return {
            "t": st.t,
            "leaves": [st.leaves[i] for i in range(MAXLEV + 1)],
            "leaf_updates": st.leaf_updates,
            "near_threshold": st.near_threshold,
            "iterations": st.iterations,
            "mass": [st.mass[k] for k in range(self.m)],
        }

    def near_threshold(self, inst: int = 0):
        """Near-threshold decisions of one instance since its last load /
        set_leaves: sorted list of (iteration, level, Morton key)."""
        L = load_library()
        n = ctypes.c_int64()
        self._check(L.mr_near_threshold(self._h, inst, None, None, None, 0, ctypes.byref(n)), "mr_near_threshold")
        it = np.zeros(n.value, dtype=np.int64)
        lv = np.zeros(n.value, dtype=np.int32)
        ky = np.zeros(n.value, dtype=np.uint64)
        if n.value:
            self._check(L.mr_near_threshold(self._h, inst, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ky.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n.value,
                                            ctypes.byref(n)), "mr_near_threshold")
        return [(int(a), int(b), int(c)) for a, b, c in zip(it, lv, ky)]

    def footprint(self) -> int:
        """Device bytes the context holds."""
        v = ctypes.c_size_t()
        self._check(load_library().mr_footprint(self._h, ctypes.byref(v)), "mr_footprint")
        return v.value

    def level_updates(self, inst: int = 0):
        arr = (ctypes.c_int64 * (MAXLEV + 1))()
        self._check(load_library().mr_level_updates(self._h, inst, arr), "mr_level_updates")
        return np.array(arr[:], dtype=np.int64)

    def stage_items(self):
        """Cumulative leaf-stage updates of the bulk stage kernel, stages 1-3."""
        arr = (ctypes.c_int64 * 3)()
        self._check(load_library().mr_stage_items(self._h, arr), "mr_stage_items")
        return np.array(arr[:], dtype=np.int64)

    def timing_start(self, kernel_class: str):
        self._check(load_library().mr_timing_start(self._h, KC[kernel_class]), "mr_timing_start")

    def timing_stop(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(load_library().mr_timing_stop(self._h, ctypes.byref(ms), ctypes.byref(n)), "mr_timing_stop")
        return ms.value, n.value

    def synchronize(self):
        self._check(load_library().mr_synchronize(self._h), "mr_synchronize")


class Batch:
    """Solves of uneven size under the library's scheduler (mr_batch_*):
    classes of (scheme, dim, largest finest level, slots), admission by
    device footprint, per-solve CFL steps, retirement at the final time."""

    def __init__(self, classes, hbm_budget: int, alloc: MrAlloc = None):
        """classes: list of (cfg, L_max, slots)."""
        import torch

        self.torch = torch
        L = load_library()
        arr = (MrClassDesc * len(classes))()
        self.ncomp = []
        for j, (cfg, L_max, slots) in enumerate(classes):
            arr[j].dim, arr[j].L_max, arr[j].slots = cfg["dim"], int(L_max), int(slots)
            arr[j].scheme = make_scheme(cfg)
        self._alloc = alloc
        h = ctypes.c_void_p()
        self._h = None
        rc = L.mr_batch_create(len(classes), arr, int(hbm_budget), ctypes.byref(alloc) if alloc is not None else None,
                               ctypes.byref(h))
        if rc != OK:
            raise MrError(rc, "mr_batch_create failed")
        self._h = h
        self.slots = sum(int(c[2]) for c in classes)
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            load_library().mr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            msg = load_library().mr_batch_last_error(self._h) if self._h else b""
            raise MrError(rc, f"{what} failed: {msg.decode() if msg else ''}")

    def admit(self, cfg: dict, L: int, eps: float, t_final: float, q0, cfl: float = 0.5, dt_max: float = 0.0):
        """Admit a solve (q0: [m, 2^{d L}]); its slot, or None when no slot
        or memory is free (MR_ECAPACITY)."""
        t = self.torch
        if isinstance(q0, np.ndarray):
            q0 = t.from_numpy(np.ascontiguousarray(q0, dtype=np.float64)).to("cuda")
        q0 = q0.contiguous()
        t.cuda.current_stream().synchronize()
        d = MrInstanceDesc(cfg["dim"], int(L), float(eps), float(t_final), float(cfl), float(dt_max), make_scheme(cfg))
        slot = ctypes.c_int()
        rc = load_library().mr_batch_admit(self._h, ctypes.byref(d), ctypes.c_void_p(q0.data_ptr()), ctypes.byref(slot))
        if rc == ECAPACITY:
            return None
        self._check(rc, "mr_batch_admit")
        return slot.value

    def step(self):
        self._check(load_library().mr_batch_step(self._h), "mr_batch_step")

    def poll(self):
        arr = (ctypes.c_int * self.slots)()
        n = ctypes.c_int()
        self._check(load_library().mr_batch_poll(self._h, arr, self.slots, ctypes.byref(n)), "mr_batch_poll")
        return list(arr[:n.value])

    def slot_info(self, slot: int):
        st, tt, ms = ctypes.c_int(), ctypes.c_double(), ctypes.c_int64()
        self._check(load_library().mr_batch_slot_info(self._h, slot, ctypes.byref(st), ctypes.byref(tt),
                                                      ctypes.byref(ms)), "mr_batch_slot_info")
        return {"state": st.value, "t": tt.value, "macro_steps": ms.value}

    def get_leaves(self, slot: int, m: int):
        L = load_library()
        n = ctypes.c_int64()
        self._check(L.mr_batch_get_leaves(self._h, slot, None, None, 0, ctypes.byref(n)), "mr_batch_get_leaves")
        keys = np.zeros(n.value, dtype=np.uint64)
        q = np.zeros((m, n.value))
        self._check(L.mr_batch_get_leaves(self._h, slot, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
                                          ctypes.byref(n)), "mr_batch_get_leaves")
        return keys, q

    def release(self, slot: int):
        self._check(load_library().mr_batch_release(self._h, slot), "mr_batch_release")

    def footprint(self) -> int:
        v = ctypes.c_size_t()
        self._check(load_library().mr_batch_footprint(self._h, ctypes.byref(v)), "mr_batch_footprint")
        return v.value
