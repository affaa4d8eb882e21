"""Python binding of libbhmc.so (ctypes).

Argument marshalling only: every step of the treecode path runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.  If
the library is missing the import of this module succeeds but every call
raises, so that a missing build can never be mistaken for a result.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BHMC_LIB") or os.path.join(_HERE, "libbhmc.so")

BHMC_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EOUTSIDE", -3: "EOVERLAP", -4: "ENOMEM", -5: "EHIP",
                -6: "ECAPACITY", -7: "ESTACK", -8: "EINTERNAL"}
REASON_NONE, REASON_WALL, REASON_OVERLAP = 0, 1, 2


class Params(C.Structure):
    _fields_ = [
        ("l_B", C.c_double), ("theta", C.c_double),
        ("p", C.c_int32), ("leaf_cap", C.c_int32), ("n0", C.c_int32), ("max_depth", C.c_int32),
        ("geom", C.c_int32), ("images", C.c_int32),
        ("box_lo", C.c_double * 3), ("box_side", C.c_double),
        ("a", C.c_double), ("Q_center", C.c_double), ("eps_in", C.c_double), ("eps_out", C.c_double),
        ("r_min", C.c_double), ("r_max", C.c_double), ("hard_core", C.c_double),
        ("slot_slack", C.c_int32), ("far_fp32", C.c_int32), ("line_images", C.c_int32), ("reserved", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [("moves", C.c_int64), ("accepted", C.c_int64), ("rejected_wall", C.c_int64),
                ("rejected_overlap", C.c_int64), ("rejected_metropolis", C.c_int64),
                ("rebuilds", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n", "nsrc", "ncell", "nleaf", "nterms", "depth", "pool")]


class BhmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None
_v = C.c_void_p
_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_u64 = C.POINTER(C.c_uint64)

SIGNATURES = {
    "bhmc_build": [C.POINTER(Params), C.c_int64, _v, _v, _v, _v, _v, C.POINTER(_v)],
    "bhmc_batch_create": [C.POINTER(Params), C.c_int32, C.POINTER(C.c_int64), _v, _v, _v, _v, _v,
                          C.POINTER(_v)],
    "bhmc_free": [_v],
    "bhmc_replicas": [_v],
    "bhmc_info_get": [_v, C.c_int32, C.POINTER(Info)],
    "bhmc_energy": [_v, C.c_int32, _d, _v],
    "bhmc_energy_noalloc": [_v, C.c_int32, _v, _v],
    "bhmc_delta_energy": [_v, C.c_int64, _d, _d, _i32],
    "bhmc_commit_move": [_v, C.c_int64, _d],
    "bhmc_mc_run": [_v, C.c_int32, C.c_uint64, C.c_uint64, C.c_int64, C.c_double, _v, C.POINTER(Stats)],
    "bhmc_batch_sweep": [_v, C.c_uint64, C.c_int32, C.c_double, C.c_int32, C.POINTER(Stats)],
    "bhmc_batch_autotune": [_v, C.c_uint64, C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float)],
    "bhmc_set_launch_shape": [_v, C.c_int32],
    "bhmc_energy_grad": [_v, C.c_int32, _v, _v, _d],
    "bhmc_set_frontier_capacity": [_v, C.c_int32, C.c_int32],
    "bhmc_set_moves_per_round": [_v, C.c_int32, C.POINTER(C.c_int32)],
    "bhmc_phase_ticks": [_v, C.POINTER(C.c_uint64), C.c_int32, C.c_int32, C.POINTER(C.c_int32)],
    "bhmc_get_state": [_v, C.c_int32, _v, _v, _v, _v],
    "bhmc_rebuild": [_v, C.c_int32],
    "bhmc_refresh_moments": [_v, C.c_int32],
    "bhmc_get_sorted": [_v, C.c_int32, _u64, _i32],
    "bhmc_get_cells": [_v, C.c_int32, _i32, _u64, _i32, _i32, _d, _d],
    "bhmc_get_leaves": [_v, C.c_int32, _i32, _i32, _i32, _i32, _i32],
    "bhmc_get_slots": [_v, C.c_int32, _i32],
    "bhmc_last_error": [],
}
# symbols include/bhmc.h declares (checked by the CPU test-suite)
EXPORTED = sorted(SIGNATURES)


def lib():
    """Load libbhmc.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbhmc.so is not built (run __graft_entry__.build() or "
                               "python paper_1305_1825_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            if name == "bhmc_last_error":
                f.restype = C.c_char_p
            elif name == "bhmc_free":
                f.restype = None
            else:
                f.restype = C.c_int
        _lib = L
    return _lib


def _check(st, what):
    if st != BHMC_OK:
        raise BhmcError(st, "%s: %s" % (what, lib().bhmc_last_error().decode()))


def make_params(d: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        if name in ("far_fp32", "line_images", "reserved"):
            setattr(p, name, int(d.get(name, 0)))
            continue
        if name == "box_lo":
            p.box_lo[:] = [float(v) for v in d["box_lo"]]
        else:
            setattr(p, name, d[name])
    return p


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required")
    return torch


def _dev(a, torch, device):
    t = torch.as_tensor(np.asarray(a, dtype=np.float64) if not torch.is_tensor(a) else a)
    return t.to(device=device, dtype=torch.float64).contiguous()


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Tree:
    """One or more replicas, each with its own octree, behind one library handle."""

    def __init__(self, params, x=None, y=None, z=None, q=None, *, n_per_replica=None, device="cuda:0"):
        torch = _torch()
        self.device = torch.device(device)
        plist = params if isinstance(params, (list, tuple)) else [params]
        self.params = [dict(p) for p in plist]
        xs, ys, zs, qs = (_dev(a, torch, self.device) for a in (x, y, z, q))
        self._keep = (xs, ys, zs, qs)
        h = C.c_void_p()
        if n_per_replica is None:
            pp = make_params(self.params[0])
            st = lib().bhmc_build(C.byref(pp), xs.numel(), xs.data_ptr(), ys.data_ptr(), zs.data_ptr(),
                                  qs.data_ptr(), _stream(torch), C.byref(h))
            self.n_per = [xs.numel()]
        else:
            R = len(n_per_replica)
            if len(self.params) == 1:
                self.params = self.params * R
            arr = (Params * R)(*[make_params(p) for p in self.params])
            npr = (C.c_int64 * R)(*[int(v) for v in n_per_replica])
            st = lib().bhmc_batch_create(arr, R, npr, xs.data_ptr(), ys.data_ptr(), zs.data_ptr(),
                                         qs.data_ptr(), _stream(torch), C.byref(h))
            self.n_per = [int(v) for v in n_per_replica]
        _check(st, "build")
        self.h = h
        self._keep = None

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().bhmc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def replicas(self):
        return lib().bhmc_replicas(self.h)

    def info(self, replica=0):
        inf = Info()
        _check(lib().bhmc_info_get(self.h, replica, C.byref(inf)), "info")
        return {k: int(getattr(inf, k)) for k, _ in Info._fields_}

    # ---------------------------------------------------------------- evaluation
    def energy(self, with_phi=False, replica=0):
        torch = _torch()
        E = C.c_double()
        phi = torch.empty(self.n_per[replica], dtype=torch.float64, device=self.device) if with_phi else None
        _check(lib().bhmc_energy(self.h, replica, C.byref(E), phi.data_ptr() if with_phi else None), "energy")
        return (E.value, phi) if with_phi else E.value

    def energy_noalloc(self, E_out, phi_out=None, replica=0):
        """Energy into the device tensor E_out (one float64) without allocation or
        synchronisation; phi_out (optional, n float64 on the device) gets phi_i."""
        _check(lib().bhmc_energy_noalloc(self.h, replica, E_out.data_ptr(),
                                         phi_out.data_ptr() if phi_out is not None else None), "energy_noalloc")

    def delta_energy(self, i, r_new):
        rn = (C.c_double * 3)(*[float(v) for v in r_new])
        dE = C.c_double()
        reason = C.c_int32()
        _check(lib().bhmc_delta_energy(self.h, int(i), rn, C.byref(dE), C.byref(reason)), "delta_energy")
        return dE.value, reason.value

    def commit_move(self, i, r_new):
        rn = (C.c_double * 3)(*[float(v) for v in r_new])
        _check(lib().bhmc_commit_move(self.h, int(i), rn), "commit_move")

    def mc_run(self, seed, n_moves, step, move0=0, replica=0, accept_bits=False):
        torch = _torch()
        st = Stats()
        bits = torch.zeros(n_moves, dtype=torch.uint8, device=self.device) if accept_bits else None
        _check(lib().bhmc_mc_run(self.h, replica, seed, move0, n_moves, step,
                                 bits.data_ptr() if accept_bits else None, C.byref(st)), "mc_run")
        out = st.as_dict()
        if accept_bits:
            out["accept"] = bits
        return out

    def batch_sweep(self, seed, n_sweeps, step, use_graph=True):
        R = self.replicas
        st = (Stats * R)()
        _check(lib().bhmc_batch_sweep(self.h, seed, n_sweeps, step, 1 if use_graph else 0, st), "batch_sweep")
        return [s.as_dict() for s in st]

    SHAPES = ("512 threads, 1 per CU", "256 threads, 1 per CU", "256 threads, 2 per CU")

    def autotune(self, seed=0, step=1.0, trial_moves=256):
        """Pick the Metropolis kernel's launch shape and traversal tile (trial moves per
        round) by timing each candidate on the replicas as built; leaves them as built.
        Returns the choice (3 shape + tile), the shape, the moves per round kept and
        every candidate's ms (0: not tried)."""
        choice = C.c_int32()
        ms = (C.c_float * (3 * len(self.SHAPES)))()
        _check(lib().bhmc_batch_autotune(self.h, seed, step, trial_moves, C.byref(choice), ms), "batch_autotune")
        c = int(choice.value)
        most = self.set_moves_per_round(0)  # the tile kept is 1, most // 2 or most moves per round
        mpr = self.set_moves_per_round((1, most // 2, most)[c % 3])
        return dict(choice=c, shape=self.SHAPES[c // 3], shape_index=c // 3, moves_per_round=mpr,
                    ms=[float(v) for v in ms])

    def set_shape(self, shape):
        _check(lib().bhmc_set_launch_shape(self.h, int(shape)), "set_launch_shape")

    def energy_grad(self, replica=0):
        torch = _torch()
        n = self.n_per[replica]
        g = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        gq = torch.empty(n, dtype=torch.float64, device=self.device)
        E = C.c_double()
        _check(lib().bhmc_energy_grad(self.h, replica, g.data_ptr(), gq.data_ptr(), C.byref(E)), "energy_grad")
        return E.value, g, gq

    def set_moves_per_round(self, moves=0):
        """1: one trial move at a time; 0 or more: rounds of that many (0 = the most the
        order allows).  Returns the moves per round the handle will use."""
        eff = C.c_int32()
        _check(lib().bhmc_set_moves_per_round(self.h, int(moves), C.byref(eff)), "set_moves_per_round")
        return int(eff.value)

    PHASES = ("setup", "levels", "flagged_scan", "far", "near", "overlap", "paths", "corrections", "decisions",
              "slots", "moments", "rounds", "moves", "chunks", "entries", "empty_entries", "far_entries",
              "near_entries", "hook_paths", "hook_prefetch")

    def phase_ticks(self, reset=True):
        """Phase timers of the batched kernel (a library built with phase timers), else {}."""
        arr = (C.c_uint64 * 32)()
        cnt = C.c_int32()
        _check(lib().bhmc_phase_ticks(self.h, arr, 32, 1 if reset else 0, C.byref(cnt)), "phase_ticks")
        return {self.PHASES[k]: int(arr[k]) for k in range(min(cnt.value, len(self.PHASES)))}

    def set_frontier_capacity(self, lds_entries=4096, allow_spill=True):
        _check(lib().bhmc_set_frontier_capacity(self.h, int(lds_entries), 1 if allow_spill else 0),
               "set_frontier_capacity")

    def state(self, replica=0):
        torch = _torch()
        n = self.n_per[replica]
        out = [torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(4)]
        _check(lib().bhmc_get_state(self.h, replica, *[t.data_ptr() for t in out]), "get_state")
        return out

    def refresh_moments(self, replica=0):
        _check(lib().bhmc_refresh_moments(self.h, replica), "refresh_moments")

    def rebuild(self, replica=0):
        _check(lib().bhmc_rebuild(self.h, replica), "rebuild")

    # ---------------------------------------------------------------- introspection
    def sorted(self, replica=0):
        ns = self.info(replica)["nsrc"]
        k = np.zeros(ns, np.uint64)
        p = np.zeros(ns, np.int32)
        _check(lib().bhmc_get_sorted(self.h, replica, k.ctypes.data_as(_u64), p.ctypes.data_as(_i32)), "sorted")
        return k, p

    def cells(self, replica=0, moments=True):
        inf = self.info(replica)
        nc, nt = inf["ncell"], inf["nterms"]
        lev = np.zeros(nc, np.int32); km = np.zeros(nc, np.uint64); cnt = np.zeros(nc, np.int32)
        link = np.zeros(nc, np.int32); geo = np.zeros((nc, 4))
        M = np.zeros((nc, nt)) if moments else None
        _check(lib().bhmc_get_cells(self.h, replica, lev.ctypes.data_as(_i32), km.ctypes.data_as(_u64),
                                    cnt.ctypes.data_as(_i32), link.ctypes.data_as(_i32), geo.ctypes.data_as(_d),
                                    M.ctypes.data_as(_d) if moments else None), "cells")
        return dict(level=lev, kmin=km, count=cnt, link=link, geo=geo, M=M)

    def leaves(self, replica=0):
        nl = self.info(replica)["nleaf"]
        arr = [np.zeros(nl, np.int32) for _ in range(5)]
        _check(lib().bhmc_get_leaves(self.h, replica, *[a.ctypes.data_as(_i32) for a in arr]), "leaves")
        return dict(cell=arr[0], base=arr[1], cap=arr[2], begin=arr[3], end=arr[4])

    def slots(self, replica=0):
        pool = self.info(replica)["pool"]
        s = np.zeros(pool, np.int32)
        _check(lib().bhmc_get_slots(self.h, replica, s.ctypes.data_as(_i32)), "slots")
        return s

    def leaf_members(self, replica=0):
        """Source indices of every leaf in slot order (list indexed by leaf)."""
        lv = self.leaves(replica)
        cells = self.cells(replica, moments=False)
        pool = self.slots(replica)
        return [pool[b:b + cells["count"][c]].copy() for c, b in zip(lv["cell"], lv["base"])]
