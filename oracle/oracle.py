"""ctypes wrapper around the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke`` and
the CPU-baseline leg of ``bench.py``; the GPU library never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EUNSTABLE = 0, 1, 4


def build(force=True):
    """Compile oracle.c with gcc (plain C99, no FP contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        sig = {
            "or_create": (P, [P, I32, P, P, I32]),
            "or_free": (None, [P]),
            "or_set_tree": (I32, [P, P, I64]),
            "or_tree_bits": (I64, [P, P, I64]),
            "or_n_leaves": (I64, [P]),
            "or_n_dof_per_leaf": (I32, [P]),
            "or_leaf_info": (None, [P, P, P]),
            "or_leaf_nodes": (I32, [P, P]),
            "or_set_params": (I32, [P, P, D, P]),
            "or_set_stimulus": (I32, [P, P, I32]),
            "or_set_state": (I32, [P, P, P]),
            "or_get_state": (I32, [P, P, P]),
            "or_assemble": (I32, [P]),
            "or_dense_operators": (I32, [P, P, P]),
            "or_apply_K": (I32, [P, P, P]),
            "or_step_global": (I32, [P, D, D, I64]),
            "or_cfl": (I32, [P, P]),
            "or_levels": (I32, [P, D, I32, P]),
            "or_rvt_indicator": (I32, [P, P, P, D, D, P]),
            "or_levels_cell": (I32, [P, D, I32, P, D, D, P]),
            "or_bucket": (None, [I64, P, I32, P, P]),
            "or_lts_barrier": (I32, [P, D, D, P, I32, P, I64, P, P]),
            "or_indicator": (I32, [P, P]),
            "or_adapt": (I32, [P, P, D, D, P, P]),
            "or_eval_points": (I32, [P, P, I64, P]),
            "or_element_update": (I32, [P, I64, P, D, D, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            # or_create's first arg is an int; fix below
            f.argtypes = args
        L.or_create.argtypes = [I32, I32, P, P, I32]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != OK:
        raise OracleError(f"{what} failed with code {rc}")


class Oracle:
    """One simulation in the oracle: forest mesh, parameters and state."""

    def __init__(self, dim, p, n, length, max_depth=0):
        n3 = np.ones(3, dtype=np.int32)
        l3 = np.ones(3, dtype=np.float64)
        n3[:dim] = n[:dim]
        l3[:dim] = length[:dim]
        self.dim, self.p = dim, p
        self._n3, self._l3 = n3, l3
        self.h = lib().or_create(dim, p, _p(n3), _p(l3), max_depth)
        if not self.h:
            raise OracleError("or_create rejected the mesh description")
        self.np_ = (p + 1) ** dim

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().or_free(h)
            self.h = None

    # mesh -------------------------------------------------------------
    def set_tree(self, bits):
        b = np.ascontiguousarray(bits, dtype=np.uint8)
        _check(lib().or_set_tree(self.h, _p(b), b.size), "or_set_tree")

    def tree_bits(self):
        n = lib().or_tree_bits(self.h, None, 0)
        out = np.zeros(n, dtype=np.uint8)
        lib().or_tree_bits(self.h, _p(out), n)
        return out

    @property
    def n_leaves(self):
        return lib().or_n_leaves(self.h)

    def leaf_info(self):
        E = self.n_leaves
        depth = np.zeros(E, dtype=np.int32)
        coords = np.zeros((E, 3), dtype=np.int64)
        lib().or_leaf_info(self.h, _p(depth), _p(coords))
        return depth, coords

    def leaf_nodes(self):
        out = np.zeros((self.n_leaves * self.np_, 3))
        lib().or_leaf_nodes(self.h, _p(out))
        return out

    # parameters -------------------------------------------------------
    def set_params(self, D, gamma, ap=(8.0, 0.15, 0.002, 0.2, 0.3)):
        D = np.asarray(D, dtype=np.float64)
        if D.shape != (3, 3):
            full = np.zeros((3, 3))
            full[: D.shape[0], : D.shape[1]] = D
            D = full
        D = np.ascontiguousarray(D)
        a = np.ascontiguousarray(ap, dtype=np.float64)
        _check(lib().or_set_params(self.h, _p(D), float(gamma), _p(a)), "or_set_params")

    def set_stimulus(self, boxes):
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 9))
        _check(lib().or_set_stimulus(self.h, _p(b), b.shape[0]), "or_set_stimulus")

    # state ------------------------------------------------------------
    def set_state(self, u=None, v=None):
        N = self.n_leaves * self.np_
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(N)
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64).reshape(N)
        _check(lib().or_set_state(self.h, None if uu is None else _p(uu), None if vv is None else _p(vv)),
               "or_set_state")

    def get_state(self):
        N = self.n_leaves * self.np_
        u = np.zeros(N)
        v = np.zeros(N)
        lib().or_get_state(self.h, _p(u), _p(v))
        return u, v

    # operators --------------------------------------------------------
    def dense_operators(self):
        N = self.n_leaves * self.np_
        K = np.zeros((N, N))
        M = np.zeros((N, N))
        _check(lib().or_dense_operators(self.h, _p(K), _p(M)), "or_dense_operators")
        return K, M

    def apply_K(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros_like(u)
        _check(lib().or_apply_K(self.h, _p(u), _p(out)), "or_apply_K")
        return out

    # stepping ---------------------------------------------------------
    def step_global(self, dt, t0, n_steps):
        _check(lib().or_step_global(self.h, float(dt), float(t0), int(n_steps)), "or_step_global")

    def cfl(self):
        out = np.zeros(self.n_leaves)
        _check(lib().or_cfl(self.h, _p(out)), "or_cfl")
        return out

    def levels(self, dt_barrier, n_levels):
        out = np.zeros(self.n_leaves, dtype=np.int8)
        rc = lib().or_levels(self.h, float(dt_barrier), int(n_levels), _p(out))
        if rc not in (OK, EUNSTABLE):
            _check(rc, "or_levels")
        return out, rc

    def rvt_indicator(self, u_a, v_a, t_a, t_b):
        """RV-T temporal indicator per leaf over [t_a, t_b] (current state = t_b)."""
        n = self.n_leaves * self.np_
        ua = np.ascontiguousarray(u_a, dtype=np.float64)
        va = np.ascontiguousarray(v_a, dtype=np.float64)
        assert ua.size == n and va.size == n
        out = np.zeros(self.n_leaves)
        _check(lib().or_rvt_indicator(self.h, _p(ua), _p(va), float(t_a), float(t_b), _p(out)), "or_rvt_indicator")
        return out

    def levels_cell(self, dt_barrier, n_levels, eta_t, tau_cell, dt_cell):
        out = np.zeros(self.n_leaves, dtype=np.int8)
        e = np.ascontiguousarray(eta_t, dtype=np.float64)
        rc = lib().or_levels_cell(self.h, float(dt_barrier), int(n_levels), _p(e), float(tau_cell), float(dt_cell),
                                  _p(out))
        if rc not in (OK, EUNSTABLE):
            _check(rc, "or_levels_cell")
        return out, rc

    @staticmethod
    def bucket(level, n_levels):
        level = np.ascontiguousarray(level, dtype=np.int8)
        perm = np.zeros(level.size, dtype=np.int32)
        cnt = np.zeros(n_levels, dtype=np.int32)
        lib().or_bucket(level.size, _p(level), int(n_levels), _p(perm), _p(cnt))
        return perm, cnt

    def lts_barrier(self, dt_barrier, t_n, level, mode=0, trace_cap=0):
        level = np.ascontiguousarray(level, dtype=np.int8)
        tr = np.zeros((max(trace_cap, 1), 4))
        tl = np.zeros(1, dtype=np.int64)
        nu = np.zeros(1, dtype=np.int64)
        _check(lib().or_lts_barrier(self.h, float(dt_barrier), float(t_n), _p(level), int(mode),
                                    _p(tr), int(trace_cap), _p(tl), _p(nu)), "or_lts_barrier")
        return int(nu[0]), (tr[: min(int(tl[0]), trace_cap)] if trace_cap else None)

    def indicator(self):
        out = np.zeros(self.n_leaves)
        _check(lib().or_indicator(self.h, _p(out)), "or_indicator")
        return out

    def adapt(self, eta, tau_refine, tau_coarsen):
        e = np.ascontiguousarray(eta, dtype=np.float64)
        nr = np.zeros(1, dtype=np.int64)
        nc = np.zeros(1, dtype=np.int64)
        _check(lib().or_adapt(self.h, _p(e), float(tau_refine), float(tau_coarsen), _p(nr), _p(nc)),
               "or_adapt")
        return int(nr[0]), int(nc[0])

    def eval_points(self, xyz):
        pts = np.zeros((len(xyz), 3))
        xyz = np.asarray(xyz, dtype=np.float64)
        pts[:, : xyz.shape[1]] = xyz
        out = np.zeros(len(pts))
        _check(lib().or_eval_points(self.h, _p(pts), len(pts), _p(out)), "or_eval_points")
        return out

    def element_update(self, e, u_at_t, t, dt):
        u = np.ascontiguousarray(u_at_t, dtype=np.float64)
        un = np.zeros(self.np_)
        vn = np.zeros(self.np_)
        _check(lib().or_element_update(self.h, int(e), _p(u), float(t), float(dt), _p(un), _p(vn)),
               "or_element_update")
        return un, vn
