"""ctypes front end of the CPU oracle (``bhmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
it, and it imports nothing from the product package.

Parameters are passed as a plain ``dict`` with the keys of ``ORC_PARAM_FIELDS``;
arrays are numpy float64 / int arrays on the host.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bhmc_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ORC_PARAM_FIELDS = [
    ("l_B", C.c_double), ("theta", C.c_double),
    ("p", C.c_int32), ("leaf_cap", C.c_int32), ("n0", C.c_int32), ("max_depth", C.c_int32),
    ("geom", C.c_int32), ("images", C.c_int32),
    ("box_lo", C.c_double * 3), ("box_side", C.c_double),
    ("a", C.c_double), ("Q_center", C.c_double), ("eps_in", C.c_double), ("eps_out", C.c_double),
    ("r_min", C.c_double), ("r_max", C.c_double), ("hard_core", C.c_double),
    ("slot_slack", C.c_int32), ("line_images", C.c_int32),
]


class OrcParams(C.Structure):
    _fields_ = ORC_PARAM_FIELDS


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP contraction off, see the C header)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_i32 = C.POINTER(C.c_int32)
_u64 = C.POINTER(C.c_uint64)
_u32 = C.POINTER(C.c_uint32)
_u8 = C.POINTER(C.c_uint8)
_P = C.POINTER(OrcParams)
_T = C.c_void_p


def _declare(L):
    sig = {
        "orc_philox": (None, [_u32, _u32, _u32]),
        "orc_draw_move": (None, [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64, C.c_double, _i64, _d, _d]),
        "orc_kelvin": (None, [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _d]),
        "orc_keys": (None, [_P, C.c_int64, _d, _d, _d, _u64]),
        "orc_direct_energy": (C.c_double, [_P, C.c_int64, _d, _d, _d, _d]),
        "orc_direct_delta": (C.c_double, [_P, C.c_int64, _d, _d, _d, _d, C.c_int64, _d]),
        "orc_direct_phi": (None, [_P, C.c_int64, _d, _d, _d, _d, _d]),
        "orc_direct_grad": (None, [_P, C.c_int64, _d, _d, _d, _d, _d, _d, _d, _d]),
        "orc_tree_build": (C.c_int, [_P, C.c_int64, _d, _d, _d, _d, C.POINTER(_T)]),
        "orc_tree_free": (None, [_T]),
        "orc_tree_phi": (C.c_double, [_T, _d, C.POINTER(C.c_int), C.c_int]),
        "orc_tree_phi_counts": (C.c_double, [_T, _d, C.POINTER(C.c_int), C.c_int, _i64]),
        "orc_tree_far_magnitude": (C.c_double, [_T, _d, C.POINTER(C.c_int), C.c_int]),
        "orc_tree_delta": (C.c_double, [_T, C.c_int64, _d, C.POINTER(C.c_int), _i64]),
        "orc_tree_commit": (C.c_int, [_T, C.c_int64, _d]),
        "orc_tree_energy": (C.c_double, [_T, _d]),
        "orc_tree_grad": (C.c_double, [_T, _d, _d, _d, _d]),
        "orc_mc_run": (C.c_int, [C.POINTER(_T), C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64,
                                 C.c_double, _u8, _d, _i64, _i64]),
        "orc_direct_mc_run": (C.c_int, [_P, C.c_int64, _d, _d, _d, _d, C.c_uint64, C.c_uint32,
                                        C.c_uint64, C.c_int64, C.c_double, _u8, _d, _i64]),
        "orc_tree_info": (None, [_T, _i64]),
        "orc_tree_sorted": (None, [_T, _u64, _i32]),
        "orc_tree_cells": (None, [_T, _i32, _u64, _i32, _i32, _i32, _d, _d]),
        "orc_tree_leaves": (None, [_T, _i32, _i32, _i32, _i32, _i32]),
        "orc_tree_leaf_slots": (C.c_int, [_T, C.c_int, _i32]),
        "orc_tree_tracking": (None, [_T, _i32, _i32]),
        "orc_tree_sources": (None, [_T, _d, _d, _d, _d]),
        "orc_tree_fresh_moments": (None, [_T, _d]),
        "orc_taylor": (None, [C.c_int, C.c_double, C.c_double, C.c_double, _d]),
        "orc_multi_indices": (None, [C.c_int, _i32]),
        "orc_tree_certificate": (C.c_double, [_T, _d, C.POINTER(C.c_int), C.c_int]),
        "orc_line_rule": (C.c_int, [C.c_double, C.c_int, _d, _d]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def params(d: dict) -> OrcParams:
    p = OrcParams()
    for name, _ in ORC_PARAM_FIELDS:
        if name == "line_images":
            p.line_images = int(d.get("line_images", 0))
            continue
        v = d[name]
        if name == "box_lo":
            p.box_lo[:] = [float(x) for x in v]
        else:
            setattr(p, name, v)
    return p


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def nterms(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


# ---------------------------------------------------------------- primitives
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c, _u32), _ptr(k, _u32), _ptr(out, _u32))
    return out


def draw_move(seed, replica, m, n, step):
    i = C.c_int64()
    d = np.zeros(3)
    al = C.c_double()
    lib().orc_draw_move(seed, replica, m, n, step, C.byref(i), _ptr(d, _d), C.byref(al))
    return i.value, d, al.value


def kelvin(a, gamma, x, y, z, q):
    out = np.zeros(4)
    lib().orc_kelvin(a, gamma, x, y, z, q, _ptr(out, _d))
    return out


def line_rule(sigma, M):
    """Nodes and weights of the M-point Gauss rule for the weight t^(sigma - 1) on
    [0, 1] (the line image of the multiple-image model)."""
    t = np.zeros(8)
    w = np.zeros(8)
    if lib().orc_line_rule(float(sigma), int(M), _ptr(t, _d), _ptr(w, _d)) != 0:
        raise ValueError("line rule needs 1 <= M <= 8 and 1/2 <= sigma <= 1")
    return t[:M].copy(), w[:M].copy()


def keys(P: dict, x, y, z):
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.zeros(len(x), dtype=np.uint64)
    pp = params(P)
    lib().orc_keys(C.byref(pp), len(x), _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(out, _u64))
    return out


def taylor(p, R):
    T = np.zeros(nterms(p))
    lib().orc_taylor(p, float(R[0]), float(R[1]), float(R[2]), _ptr(T, _d))
    return T


def multi_indices(p):
    out = np.zeros(3 * nterms(p), dtype=np.int32)
    lib().orc_multi_indices(p, _ptr(out, _i32))
    return out.reshape(-1, 3)


# ---------------------------------------------------------------- direct sums
def direct_energy(P, x, y, z, q):
    x, y, z, q = map(_f64, (x, y, z, q))
    pp = params(P)
    return lib().orc_direct_energy(C.byref(pp), len(x), _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(q, _d))


def direct_delta(P, x, y, z, q, i, rn):
    x, y, z, q = map(_f64, (x, y, z, q))
    r = _f64(rn)
    pp = params(P)
    return lib().orc_direct_delta(C.byref(pp), len(x), _ptr(x, _d), _ptr(y, _d), _ptr(z, _d),
                                  _ptr(q, _d), int(i), _ptr(r, _d))


def direct_phi(P, x, y, z, q):
    x, y, z, q = map(_f64, (x, y, z, q))
    out = np.zeros(len(x))
    pp = params(P)
    lib().orc_direct_phi(C.byref(pp), len(x), _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(q, _d), _ptr(out, _d))
    return out


def direct_grad(P, x, y, z, q):
    x, y, z, q = map(_f64, (x, y, z, q))
    n = len(x)
    g = [np.zeros(n) for _ in range(4)]
    pp = params(P)
    lib().orc_direct_grad(C.byref(pp), n, _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(q, _d),
                          *[_ptr(a, _d) for a in g])
    return np.stack(g[:3], axis=1), g[3]


def direct_mc_run(P, x, y, z, q, seed, replica, move0, n_moves, step):
    x, y, z, q = (np.array(a, dtype=np.float64) for a in (x, y, z, q))
    bits = np.zeros(n_moves, dtype=np.uint8)
    dE = np.zeros(n_moves)
    stats = np.zeros(5, dtype=np.int64)
    pp = params(P)
    st = lib().orc_direct_mc_run(C.byref(pp), len(x), _ptr(x, _d), _ptr(y, _d), _ptr(z, _d), _ptr(q, _d),
                                 seed, replica, move0, n_moves, step, _ptr(bits, _u8), _ptr(dE, _d),
                                 _ptr(stats, _i64))
    if st:
        raise RuntimeError("orc_direct_mc_run failed: %d" % st)
    return dict(accept=bits, dE=dE, stats=stats, x=x, y=y, z=z)


# ---------------------------------------------------------------- treecode
class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s: status %d" % (what, code))
        self.code = code


class Tree:
    """Serial CPU treecode over ions (and their Kelvin images)."""

    def __init__(self, P: dict, x, y, z, q):
        self.P = dict(P)
        self._pp = params(P)
        x, y, z, q = map(_f64, (x, y, z, q))
        h = _T()
        st = lib().orc_tree_build(C.byref(self._pp), len(x), _ptr(x, _d), _ptr(y, _d), _ptr(z, _d),
                                  _ptr(q, _d), C.byref(h))
        if st:
            raise OracleError(st, "orc_tree_build")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().orc_tree_free(h)
            self.h = None

    # introspection
    def info(self):
        a = np.zeros(6, dtype=np.int64)
        lib().orc_tree_info(self.h, _ptr(a, _i64))
        return dict(n=int(a[0]), nsrc=int(a[1]), ncell=int(a[2]), nleaf=int(a[3]),
                    nterms=int(a[4]), depth=int(a[5]))

    def sorted(self):
        ns = self.info()["nsrc"]
        k = np.zeros(ns, dtype=np.uint64)
        p = np.zeros(ns, dtype=np.int32)
        lib().orc_tree_sorted(self.h, _ptr(k, _u64), _ptr(p, _i32))
        return k, p

    def cells(self, moments=True):
        inf = self.info()
        nc, nt = inf["ncell"], inf["nterms"]
        lev = np.zeros(nc, np.int32); km = np.zeros(nc, np.uint64); cnt = np.zeros(nc, np.int32)
        isl = np.zeros(nc, np.int32); par = np.zeros(nc, np.int32); geo = np.zeros((nc, 4))
        M = np.zeros((nc, nt)) if moments else None
        lib().orc_tree_cells(self.h, _ptr(lev, _i32), _ptr(km, _u64), _ptr(cnt, _i32), _ptr(isl, _i32),
                             _ptr(par, _i32), _ptr(geo, _d), _ptr(M, _d) if moments else None)
        return dict(level=lev, kmin=km, count=cnt, is_leaf=isl, parent=par, geo=geo, M=M)

    def leaves(self):
        nl = self.info()["nleaf"]
        arr = [np.zeros(nl, np.int32) for _ in range(5)]
        lib().orc_tree_leaves(self.h, *[_ptr(a, _i32) for a in arr])
        return dict(cell=arr[0], count=arr[1], cap=arr[2], begin=arr[3], end=arr[4])

    def leaf_slots(self, l):
        lv = self.leaves()
        out = np.zeros(max(int(lv["cap"][l]), 1), np.int32)
        k = lib().orc_tree_leaf_slots(self.h, int(l), _ptr(out, _i32))
        return out[:k].copy()

    def tracking(self):
        ns = self.info()["nsrc"]
        a = np.zeros(ns, np.int32); b = np.zeros(ns, np.int32)
        lib().orc_tree_tracking(self.h, _ptr(a, _i32), _ptr(b, _i32))
        return a, b

    def sources(self):
        ns = self.info()["nsrc"]
        arr = [np.zeros(ns) for _ in range(4)]
        lib().orc_tree_sources(self.h, *[_ptr(a, _d) for a in arr])
        return arr

    def fresh_moments(self):
        inf = self.info()
        M = np.zeros((inf["ncell"], inf["nterms"]))
        lib().orc_tree_fresh_moments(self.h, _ptr(M, _d))
        return M

    # evaluation
    def phi(self, xt, exclude=()):
        r = _f64(xt)
        ex = (C.c_int * max(len(exclude), 1))(*[int(e) for e in exclude])
        return lib().orc_tree_phi(self.h, _ptr(r, _d), ex, len(exclude))

    def phi_counts(self, xt, exclude=()):
        """Potential and the traversal's counts (visited, far, near sources) for one target."""
        r = _f64(xt)
        ex = (C.c_int * max(len(exclude), 1))(*[int(e) for e in exclude])
        c = np.zeros(3, dtype=np.int64)
        v = lib().orc_tree_phi_counts(self.h, _ptr(r, _d), ex, len(exclude), _ptr(c, _i64))
        return v, c

    def far_magnitude(self, xt, exclude=()):
        """sum over the expanded cells of sum_n |T_n M'_n| at one target."""
        r = _f64(xt)
        ex = (C.c_int * max(len(exclude), 1))(*[int(e) for e in exclude])
        return lib().orc_tree_far_magnitude(self.h, _ptr(r, _d), ex, len(exclude))

    def certificate(self, xt, exclude=()):
        r = _f64(xt)
        ex = (C.c_int * max(len(exclude), 1))(*[int(e) for e in exclude])
        return lib().orc_tree_certificate(self.h, _ptr(r, _d), ex, len(exclude))

    def delta(self, i, rn, counts=False):
        r = _f64(rn)
        reason = C.c_int()
        c = np.zeros(3, dtype=np.int64)
        dE = lib().orc_tree_delta(self.h, int(i), _ptr(r, _d), C.byref(reason), _ptr(c, _i64))
        if counts:
            return dE, reason.value, c
        return dE, reason.value

    def commit(self, i, rn):
        r = _f64(rn)
        st = lib().orc_tree_commit(self.h, int(i), _ptr(r, _d))
        if st:
            raise OracleError(st, "orc_tree_commit")

    def energy(self, with_phi=False):
        n = self.info()["n"]
        phi = np.zeros(n)
        E = lib().orc_tree_energy(self.h, _ptr(phi, _d))
        return (E, phi) if with_phi else E

    def grad(self):
        n = self.info()["n"]
        g = [np.zeros(n) for _ in range(4)]
        E = lib().orc_tree_grad(self.h, *[_ptr(a, _d) for a in g])
        return E, np.stack(g[:3], axis=1), g[3]

    def mc_run(self, seed, replica, move0, n_moves, step):
        bits = np.zeros(n_moves, dtype=np.uint8)
        dE = np.zeros(n_moves)
        idx = np.zeros(n_moves, dtype=np.int64)
        stats = np.zeros(5, dtype=np.int64)
        st = lib().orc_mc_run(C.byref(self.h), seed, replica, move0, n_moves, step, _ptr(bits, _u8),
                              _ptr(dE, _d), _ptr(idx, _i64), _ptr(stats, _i64))
        if st:
            raise OracleError(st, "orc_mc_run")
        return dict(accept=bits, dE=dE, i=idx, stats=stats)
