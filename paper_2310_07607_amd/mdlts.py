"""ctypes binding of libmdlts.so (include/mdlts.h), same names as the C ABI.

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch supplies the stream and (optionally) the device memory
through its caching allocator.  There is no fallback: if the library is not
built, importing the library raises.
"""
import ctypes
import os
import re
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmdlts.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mdlts.h")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE, EBUSY = range(7)
FP64, FP32 = 0, 1
_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSTABLE", 5: "ESTATE", 6: "EBUSY"}


class MdltsError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {_NAMES.get(status, status)} ({strerror(status)})")


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("len", ctypes.c_double * 3), ("max_depth", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("precision", ctypes.c_int)]


class APParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("a", ctypes.c_double), ("eps0", ctypes.c_double),
                ("mu1", ctypes.c_double), ("mu2", ctypes.c_double)]


class StimBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("t_on", ctypes.c_double),
                ("t_off", ctypes.c_double), ("amp", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libmdlts.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2310_07607_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, S, I, D = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "mdlts_strerror": (ctypes.c_char_p, [I]),
        "mdlts_ctx_create": (I, [I, P, P, PP]),
        "mdlts_ctx_destroy": (I, [P]),
        "mdlts_sync": (I, [P]),
        "mdlts_sim_create": (I, [P, P, PP]),
        "mdlts_sim_destroy": (I, [P]),
        "mdlts_set_tree": (I, [P, P, S]),
        "mdlts_get_tree": (I, [P, P, S, P]),
        "mdlts_n_leaves": (I, [P, P]),
        "mdlts_set_conductivity": (I, [P, P, D]),
        "mdlts_set_ionic": (I, [P, P]),
        "mdlts_set_stimulus": (I, [P, P, I]),
        "mdlts_set_state": (I, [P, P, P, S]),
        "mdlts_get_state": (I, [P, P, P, S]),
        "mdlts_set_time": (I, [P, D]),
        "mdlts_assign_levels": (I, [P, D, P]),
        "mdlts_assign_uniform": (I, [P, D, I, P]),
        "mdlts_get_levels": (I, [P, P, P, P, S]),
        "mdlts_get_cfl": (I, [P, P, S]),
        "mdlts_step": (I, [P, I]),
        "mdlts_indicator": (I, [P, P, S, P]),
        "mdlts_indicator_noalloc": (I, [P, P, S, P]),
        "mdlts_adapt": (I, [P, P, S, D, D, P, P]),
        "mdlts_counters": (I, [P, P, P]),
        "mdlts_profile": (I, [P, I]),
        "mdlts_batch_step": (I, [P, P, I, I]),
        "mdlts_batch_adapt": (I, [P, P, I, D, D, P]),
        "mdlts_set_graphs": (I, [P, I]),
        "mdlts_batch_profile": (I, [P, I]),
        "mdlts_batch_profile_read": (I, [P, P, P, P, P, P]),
        "mdlts_profile_read": (I, [P, P, P, P]),
        "mdlts_cfl_bound": (I, [P, P, D, I, P]),
        "mdlts_plan_adapt": (I, [P, P, S, P, S, D, D, P, S, P]),
        "mdlts_plan_levels": (I, [P, P, S, P, D, D, P, P, P, P, S]),
        "mdlts_memory_bound": (I, [P, ctypes.c_int64, P]),
        "mdlts_rvt_snapshot": (I, [P]),
        "mdlts_assign_levels_auto": (I, [P, P, P]),
        "mdlts_rvt_indicator": (I, [P, P, S, P]),
        "mdlts_assign_levels_cell": (I, [P, D, D, D, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(status):
    try:
        return lib().mdlts_strerror(int(status)).decode()
    except Exception:  # pragma: no cover
        return "?"


def declared_symbols(header=HEADER):
    """Names of the functions declared in include/mdlts.h."""
    with open(header) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mdlts_[a-z_0-9]+)\s*\(", text)))


def _chk(status, what):
    if status != OK:
        raise MdltsError(status, what)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_desc(dim, order, n, length, max_depth=0, n_levels=1, precision="f64"):
    d = MeshDesc()
    d.dim, d.order = int(dim), int(order)
    for k in range(3):
        d.n[k] = int(n[k]) if k < len(n) and k < dim else 1
        d.len[k] = float(length[k]) if k < len(length) and k < dim else 1.0
    d.max_depth, d.n_levels = int(max_depth), int(n_levels)
    d.precision = FP32 if precision in ("f32", FP32, "fp32") else FP64
    return d


def _dsym(D):
    D = np.asarray(D, dtype=np.float64)
    if D.ndim == 1:
        out = np.zeros(6)
        out[: D.size] = D
        return out
    full = np.zeros((3, 3))
    full[: D.shape[0], : D.shape[1]] = D
    return np.array([full[0, 0], full[1, 1], full[2, 2], full[0, 1], full[0, 2], full[1, 2]])


class Context:
    """A device + stream; device memory from torch's caching allocator."""

    def __init__(self, device=0, stream=None, torch_allocator=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the mdlts library runs on an MI355X only")
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._torch_stream = stream
        sptr = ctypes.c_void_p(stream.cuda_stream)
        self._alloc = None
        aptr = None
        if torch_allocator:
            dev = self.device

            def _a(nbytes, st, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
                except Exception:
                    return None

            def _f(ptr, st, user):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:  # interpreter shutdown
                    pass

            self._alloc = Allocator(ALLOC_FN(_a), FREE_FN(_f), None)
            aptr = ctypes.cast(ctypes.pointer(self._alloc), ctypes.c_void_p)
        h = ctypes.c_void_p()
        _chk(lib().mdlts_ctx_create(self.device, sptr, aptr, ctypes.byref(h)), "mdlts_ctx_create")
        self.h = h
        self._sims = weakref.WeakSet()

    def sync(self):
        _chk(lib().mdlts_sync(self.h), "mdlts_sync")

    def batch_step(self, sims, n_barriers=1):
        """Advance several simulations together (one launch per substep and kind)."""
        arr = (ctypes.c_void_p * len(sims))(*[s.h.value for s in sims])
        _chk(lib().mdlts_batch_step(self.h, arr, len(sims), int(n_barriers)), "mdlts_batch_step")

    def batch_adapt(self, sims, tau_refine, tau_coarsen, dt_barrier):
        """Indicator, adaptation and levels of several simulations with two
        synchronisations in all; dt_barrier: one per simulation."""
        arr = (ctypes.c_void_p * len(sims))(*[s.h.value for s in sims])
        dts = np.ascontiguousarray(dt_barrier, dtype=np.float64)
        if dts.size != len(sims):
            raise ValueError("one dt_barrier per simulation")
        _chk(lib().mdlts_batch_adapt(self.h, arr, len(sims), float(tau_refine), float(tau_coarsen), _p(dts)),
             "mdlts_batch_adapt")

    def set_graphs(self, enable=True):
        _chk(lib().mdlts_set_graphs(self.h, 1 if enable else 0), "mdlts_set_graphs")

    def batch_profile(self, enable=True):
        _chk(lib().mdlts_batch_profile(self.h, 1 if enable else 0), "mdlts_batch_profile")

    def batch_profile_read(self):
        """(kernel ms, launches, DoF-updates, threads per block, 0 (one block per tile))."""
        ms = ctypes.c_double()
        nl, nd = ctypes.c_uint64(), ctypes.c_uint64()
        blk, pcu = ctypes.c_int(), ctypes.c_int()
        _chk(lib().mdlts_batch_profile_read(self.h, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(nd),
                                            ctypes.byref(blk), ctypes.byref(pcu)), "mdlts_batch_profile_read")
        return ms.value, nl.value, nd.value, blk.value, pcu.value

    def close(self):
        """Destroys the context after closing every simulation created on it."""
        if getattr(self, "h", None):
            for sim in list(self._sims):
                sim.close()
            _chk(lib().mdlts_ctx_destroy(self.h), "mdlts_ctx_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation:
    """One monodomain simulation on the device (mdlts_sim)."""

    def __init__(self, ctx, dim, order, n, length, max_depth=0, n_levels=1, precision="f64"):
        self.ctx = ctx
        self.desc = make_desc(dim, order, n, length, max_depth, n_levels, precision)
        self.dim, self.order, self.n_levels = dim, order, n_levels
        self.np_ = (order + 1) ** dim
        h = ctypes.c_void_p()
        if not getattr(ctx, "h", None):
            raise RuntimeError("context is closed")
        _chk(lib().mdlts_sim_create(ctx.h, ctypes.byref(self.desc), ctypes.byref(h)), "mdlts_sim_create")
        self.h = h
        ctx._sims.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib().mdlts_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # mesh ---------------------------------------------------------------
    def set_tree(self, bits):
        b = np.ascontiguousarray(bits, dtype=np.uint8)
        _chk(lib().mdlts_set_tree(self.h, _p(b), b.size), "mdlts_set_tree")

    def get_tree(self):
        n = ctypes.c_size_t()
        _chk(lib().mdlts_get_tree(self.h, None, 0, ctypes.byref(n)), "mdlts_get_tree")
        out = np.zeros(n.value, dtype=np.uint8)
        _chk(lib().mdlts_get_tree(self.h, _p(out), out.size, ctypes.byref(n)), "mdlts_get_tree")
        return out

    @property
    def n_leaves(self):
        n = ctypes.c_size_t()
        _chk(lib().mdlts_n_leaves(self.h, ctypes.byref(n)), "mdlts_n_leaves")
        return n.value

    @property
    def n_dof(self):
        return self.n_leaves * self.np_

    # parameters ---------------------------------------------------------
    def set_conductivity(self, D, gamma):
        d = _dsym(D)
        _chk(lib().mdlts_set_conductivity(self.h, _p(d), float(gamma)), "mdlts_set_conductivity")

    def set_ionic(self, k=8.0, a=0.15, eps0=0.002, mu1=0.2, mu2=0.3):
        p = APParams(k, a, eps0, mu1, mu2)
        _chk(lib().mdlts_set_ionic(self.h, ctypes.byref(p)), "mdlts_set_ionic")

    def set_stimulus(self, boxes):
        """boxes: array [n, 9] (lo3, hi3, t_on, t_off, amp)."""
        b = np.asarray(boxes, dtype=np.float64).reshape(-1, 9)
        arr = (StimBox * max(1, len(b)))()
        for i, row in enumerate(b):
            for k in range(3):
                arr[i].lo[k], arr[i].hi[k] = row[k], row[3 + k]
            arr[i].t_on, arr[i].t_off, arr[i].amp = row[6], row[7], row[8]
        _chk(lib().mdlts_set_stimulus(self.h, arr, len(b)), "mdlts_set_stimulus")

    # state ----------------------------------------------------------------
    def set_state(self, u=None, v=None):
        N = self.n_dof
        uu = None if u is None else _f64(u, N)
        vv = None if v is None else _f64(v, N)
        _chk(lib().mdlts_set_state(self.h, None if uu is None else _p(uu), None if vv is None else _p(vv), N),
             "mdlts_set_state")

    def get_state(self):
        N = self.n_dof
        u = np.zeros(N)
        v = np.zeros(N)
        _chk(lib().mdlts_get_state(self.h, _p(u), _p(v), N), "mdlts_get_state")
        return u, v

    def set_time(self, t):
        _chk(lib().mdlts_set_time(self.h, float(t)), "mdlts_set_time")

    # levels and stepping --------------------------------------------------
    def assign_levels(self, dt_barrier):
        hist = np.zeros(self.n_levels, dtype=np.int32)
        _chk(lib().mdlts_assign_levels(self.h, float(dt_barrier), _p(hist)), "mdlts_assign_levels")
        return hist

    def assign_uniform(self, dt_barrier, level=0):
        """Every leaf on `level` (level 0: the plain global step dt_barrier)."""
        hist = np.zeros(self.n_levels, dtype=np.int32)
        _chk(lib().mdlts_assign_uniform(self.h, float(dt_barrier), int(level), _p(hist)), "mdlts_assign_uniform")
        return hist

    def assign_levels_auto(self):
        """(dt_barrier, level histogram): the largest barrier step that keeps
        every current leaf within the configured levels."""
        dt = ctypes.c_double()
        hist = np.zeros(self.n_levels, dtype=np.int32)
        _chk(lib().mdlts_assign_levels_auto(self.h, ctypes.byref(dt), _p(hist)), "mdlts_assign_levels_auto")
        return dt.value, hist

    def rvt_snapshot(self):
        """Start of the interval the RV-T temporal indicator covers."""
        _chk(lib().mdlts_rvt_snapshot(self.h), "mdlts_rvt_snapshot")

    def rvt_indicator(self, download=True):
        """(eta_t per leaf or None, max eta_t) over [snapshot time, now]."""
        m = ctypes.c_double()
        if not download:
            _chk(lib().mdlts_rvt_indicator(self.h, None, 0, ctypes.byref(m)), "mdlts_rvt_indicator")
            return None, m.value
        eta = np.zeros(self.n_leaves)
        _chk(lib().mdlts_rvt_indicator(self.h, _p(eta), eta.size, ctypes.byref(m)), "mdlts_rvt_indicator")
        return eta, m.value

    def assign_levels_cell(self, dt_barrier, tau_cell, dt_cell):
        """Levels from max(b^CFL, b^cell) with the last RV-T indicator."""
        hist = np.zeros(self.n_levels, dtype=np.int32)
        _chk(lib().mdlts_assign_levels_cell(self.h, float(dt_barrier), float(tau_cell), float(dt_cell), _p(hist)),
             "mdlts_assign_levels_cell")
        return hist

    def get_levels(self):
        E = self.n_leaves
        level = np.zeros(E, dtype=np.int8)
        perm = np.zeros(E, dtype=np.int32)
        cnt = np.zeros(self.n_levels, dtype=np.int32)
        _chk(lib().mdlts_get_levels(self.h, _p(level), _p(perm), _p(cnt), E), "mdlts_get_levels")
        return level, perm, cnt

    def get_cfl(self):
        out = np.zeros(self.n_leaves)
        _chk(lib().mdlts_get_cfl(self.h, _p(out), out.size), "mdlts_get_cfl")
        return out

    def step(self, n_barriers=1):
        _chk(lib().mdlts_step(self.h, int(n_barriers)), "mdlts_step")

    def indicator(self, download=True):
        """(eta per leaf or None, max eta); the values stay on the device for adapt()."""
        m = ctypes.c_double()
        if not download:
            _chk(lib().mdlts_indicator(self.h, None, 0, ctypes.byref(m)), "mdlts_indicator")
            return None, m.value
        eta = np.zeros(self.n_leaves)
        _chk(lib().mdlts_indicator(self.h, _p(eta), eta.size, ctypes.byref(m)), "mdlts_indicator")
        return eta, m.value

    def indicator_noalloc(self, download=True):
        """(eta per leaf or None, max eta) through the allocation-free entry
        point (fixed per-device scratch; nothing kept for adapt())."""
        m = ctypes.c_double()
        if not download:
            _chk(lib().mdlts_indicator_noalloc(self.h, None, 0, ctypes.byref(m)), "mdlts_indicator_noalloc")
            return None, m.value
        eta = np.zeros(self.n_leaves)
        _chk(lib().mdlts_indicator_noalloc(self.h, _p(eta), eta.size, ctypes.byref(m)), "mdlts_indicator_noalloc")
        return eta, m.value

    def adapt(self, tau_refine, tau_coarsen, eta=None):
        nr, nc = ctypes.c_int64(), ctypes.c_int64()
        if eta is None:
            st = lib().mdlts_adapt(self.h, None, 0, float(tau_refine), float(tau_coarsen), ctypes.byref(nr),
                                   ctypes.byref(nc))
        else:
            e = _f64(eta)
            st = lib().mdlts_adapt(self.h, _p(e), e.size, float(tau_refine), float(tau_coarsen), ctypes.byref(nr),
                                   ctypes.byref(nc))
        _chk(st, "mdlts_adapt")
        return nr.value, nc.value

    def profile(self, enable=True):
        _chk(lib().mdlts_profile(self.h, 1 if enable else 0), "mdlts_profile")

    def profile_read(self):
        """(substep kernel ms, launches, DoF-updates) since the last read."""
        ms = ctypes.c_double()
        nl, nd = ctypes.c_uint64(), ctypes.c_uint64()
        _chk(lib().mdlts_profile_read(self.h, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(nd)),
             "mdlts_profile_read")
        return ms.value, nl.value, nd.value

    def counters(self):
        n = ctypes.c_uint64()
        t = ctypes.c_double()
        _chk(lib().mdlts_counters(self.h, ctypes.byref(n), ctypes.byref(t)), "mdlts_counters")
        return n.value, t.value


# host-only planning utilities ---------------------------------------------
def cfl_bound(desc, D, gamma, depth):
    out = ctypes.c_double()
    d = _dsym(D)
    _chk(lib().mdlts_cfl_bound(ctypes.byref(desc), _p(d), float(gamma), int(depth), ctypes.byref(out)),
         "mdlts_cfl_bound")
    return out.value


def plan_adapt(desc, bits, eta, tau_refine, tau_coarsen):
    b = np.ascontiguousarray(bits, dtype=np.uint8)
    e = _f64(eta)
    n = ctypes.c_size_t()
    _chk(lib().mdlts_plan_adapt(ctypes.byref(desc), _p(b), b.size, _p(e), e.size, float(tau_refine),
                                float(tau_coarsen), None, 0, ctypes.byref(n)), "mdlts_plan_adapt")
    out = np.zeros(n.value, dtype=np.uint8)
    _chk(lib().mdlts_plan_adapt(ctypes.byref(desc), _p(b), b.size, _p(e), e.size, float(tau_refine),
                                float(tau_coarsen), _p(out), out.size, ctypes.byref(n)), "mdlts_plan_adapt")
    return out


def memory_bound(desc, max_leaves):
    """Device bytes a simulation of this shape holds with at most max_leaves leaves."""
    out = ctypes.c_uint64()
    _chk(lib().mdlts_memory_bound(ctypes.byref(desc), int(max_leaves), ctypes.byref(out)), "mdlts_memory_bound")
    return out.value


def max_leaves(desc):
    """Leaves of the forest with every root refined to max_depth."""
    roots = desc.n[0] * desc.n[1] * (desc.n[2] if desc.dim == 3 else 1)
    return roots << (desc.dim * desc.max_depth)


def plan_levels(desc, bits, n_leaves, D, gamma, dt_barrier):
    """Returns (level, perm, cnt_ge, cfl, status) computed on the host."""
    b = np.ascontiguousarray(bits, dtype=np.uint8)
    d = _dsym(D)
    level = np.zeros(n_leaves, dtype=np.int8)
    perm = np.zeros(n_leaves, dtype=np.int32)
    cnt = np.zeros(desc.n_levels, dtype=np.int32)
    cfl = np.zeros(n_leaves)
    st = lib().mdlts_plan_levels(ctypes.byref(desc), _p(b), b.size, _p(d), float(gamma), float(dt_barrier),
                                 _p(level), _p(perm), _p(cnt), _p(cfl), n_leaves)
    if st not in (OK, EUNSTABLE):
        _chk(st, "mdlts_plan_levels")
    return level, perm, cnt, cfl, st
