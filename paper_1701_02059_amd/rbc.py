"""Python binding of librbc (include/rbc.h): argument marshalling only.

Every step of the force / cell-update / time-step path runs in the HIP library;
this module passes torch device pointers and the current HIP stream through the
C ABI and raises on any status other than RBC_OK.  Importing it fails loudly if
the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbc.so")

RBC_OK, RBC_ERR_INVALID_ARG, RBC_ERR_OUT_OF_MEMORY, RBC_ERR_HIP, RBC_ERR_NOT_READY = 0, 1, 2, 3, 4
RBC_ERR_CAPACITY, RBC_ERR_NONFINITE, RBC_ERR_UNSUPPORTED, RBC_ERR_SKIN = 5, 6, 7, 8
RBC_FP64, RBC_MIXED = 0, 1

FUNCTIONS = [
    "rbc_create", "rbc_set_system", "rbc_update_cells", "rbc_forces", "rbc_step", "rbc_get_state",
    "rbc_get_pairs", "rbc_energy", "rbc_stats", "rbc_get_cells", "rbc_force_timing", "rbc_sync", "rbc_destroy",
    "rbc_status_string", "rbc_last_error", "rbc_ensemble_create", "rbc_ensemble_footprint", "rbc_ensemble_admit",
    "rbc_ensemble_step", "rbc_ensemble_get_state", "rbc_ensemble_energy", "rbc_ensemble_retire",
    "rbc_ensemble_info", "rbc_debug_array", "rbc_set_graphs", "rbc_ensemble_stage", "rbc_ensemble_commit",
    "rbc_get_pairs_noalloc", "rbc_ensemble_failed", "rbc_step_times", "rbc_host_times",
    "rbc_build_timing",
]


class RbcParams(C.Structure):
    _fields_ = [("rc", (C.c_double * 3) * 3), ("eps", C.c_double), ("zeta", C.c_double), ("mu", C.c_double),
                ("sin_theta0", C.c_double), ("r_min", C.c_double), ("wca_eps", C.c_double),
                ("wca_sigma", C.c_double), ("k_bond", C.c_double), ("mass", C.c_double * 3),
                ("inertia", C.c_double), ("cell_target", C.c_int32), ("update_every", C.c_int32),
                ("skin", C.c_double), ("lloyd_iters", C.c_int32), ("precision", C.c_int32),
                ("protein_cells", C.c_int32),
                ("vol_k", C.c_double), ("vol_target", C.c_double), ("lipid_area", C.c_double),
                ("kT", C.c_double), ("gamma", C.c_double), ("gamma_rot", C.c_double), ("seed", C.c_uint64),
                ("quench_max", C.c_double), ("quench", C.c_int32), ("inner_skin", C.c_double)]


class RbcError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(text)
        self.status = status


_lib = None


def lib():
    """Load librbc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1701_02059_amd.build.build()")
        # torch bundles its own HIP runtime under the same soname; load and initialise it
        # first so that librbc binds to that single runtime in this process
        import torch
        torch.cuda.is_available()
        L = C.CDLL(LIB_PATH)
        vp, dp, ip, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        h = C.c_void_p
        pp = C.POINTER(RbcParams)
        sig = {
            "rbc_create": [pp, vp, C.POINTER(h)],
            "rbc_set_system": [h, C.c_int64, vp, vp, vp, vp, vp, C.c_int64, vp, vp, dp, ip],
            "rbc_update_cells": [h, C.c_int32],
            "rbc_forces": [h, vp, vp, vp],
            "rbc_step": [h, C.c_int64, C.c_double],
            "rbc_get_state": [h, vp, vp, vp, vp],
            "rbc_get_pairs": [h, C.c_int64, ip, i64p],
            "rbc_get_pairs_noalloc": [h, C.c_int64, ip, i64p],
            "rbc_ensemble_failed": [h, C.c_int64, ip, ip, i64p],
            "rbc_step_times": [h, C.c_int32, C.c_int64, dp, i64p, dp],
            "rbc_host_times": [h, dp, dp],
            "rbc_build_timing": [h, dp, i64p],
            "rbc_energy": [h, dp],
            "rbc_stats": [h, i64p],
            "rbc_get_cells": [h, ip, dp],
            "rbc_force_timing": [h, C.c_int32, dp, i64p],
            "rbc_sync": [h],
            "rbc_destroy": [h],
            "rbc_ensemble_create": [pp, vp, C.c_int32, C.c_int64, C.POINTER(h)],
            "rbc_ensemble_footprint": [h, C.c_int64, C.c_int64, C.c_int64, i64p],
            "rbc_ensemble_admit": [h, C.c_int64, vp, vp, vp, vp, vp, C.c_int64, vp, vp, dp, ip, ip],
            "rbc_ensemble_stage": [h, C.c_int64, vp, vp, vp, vp, vp, C.c_int64, vp, vp, dp, ip, ip],
            "rbc_ensemble_commit": [h, C.c_int64, ip, i64p],
            "rbc_ensemble_step": [h, C.c_int64, C.c_double],
            "rbc_ensemble_get_state": [h, C.c_int32, vp, vp, vp, vp],
            "rbc_ensemble_energy": [h, C.c_int32, dp],
            "rbc_ensemble_retire": [h, C.c_int32],
            "rbc_ensemble_info": [h, i64p],
            "rbc_debug_array": [h, C.c_int32, C.c_int64, vp, i64p],
            "rbc_set_graphs": [h, C.c_int32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.rbc_status_string.argtypes = [C.c_int]
        L.rbc_status_string.restype = C.c_char_p
        L.rbc_last_error.argtypes = [h]
        L.rbc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def make_params(mp, precision: int = RBC_FP64) -> RbcParams:
    p = RbcParams()
    rc = mp.rc_table()
    for a in range(3):
        for b in range(3):
            p.rc[a][b] = float(rc[a, b])
    p.eps, p.zeta, p.mu, p.sin_theta0, p.r_min = mp.eps, float(mp.zeta), mp.mu, mp.sin_theta0, mp.r_min
    p.wca_eps, p.wca_sigma, p.k_bond = mp.wca_eps, mp.wca_sigma, mp.k_bond
    for a in range(3):
        p.mass[a] = float(mp.mass[a])
    p.inertia = mp.inertia
    p.cell_target, p.update_every, p.skin = int(mp.cell_target), int(mp.update_every), float(mp.skin)
    p.lloyd_iters, p.precision = int(mp.lloyd_iters), int(precision)
    p.protein_cells = int(getattr(mp, "protein_cells", 0))
    p.vol_k, p.vol_target = float(mp.vol_k), float(mp.vol_target)
    p.lipid_area = float(mp.lipid_area)
    p.kT, p.gamma, p.gamma_rot, p.seed = float(mp.kT), float(mp.gamma), float(mp.gamma_rot), int(mp.seed)
    p.quench, p.quench_max = int(getattr(mp, "quench", 0)), float(getattr(mp, "quench_max", 0.05))
    p.inner_skin = float(getattr(mp, "inner_skin", 0.0))
    return p


def _check(handle, status: int):
    if status != RBC_OK:
        L = lib()
        text = L.rbc_status_string(status).decode()
        if handle:
            text += ": " + L.rbc_last_error(handle).decode()
        raise RbcError(status, text)


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class _Uploaded:
    """System arrays as torch device tensors (kept alive across the call)."""

    def __init__(self, system, device="cuda"):
        import torch
        f64 = dict(dtype=torch.float64, device=device)
        self.n = system.N
        self.x = torch.as_tensor(np.ascontiguousarray(system.x), **f64)
        self.nrm = torch.as_tensor(np.ascontiguousarray(system.n), **f64)
        self.v = torch.as_tensor(np.ascontiguousarray(system.v), **f64)
        self.w = torch.as_tensor(np.ascontiguousarray(system.w), **f64)
        self.type = torch.as_tensor(np.ascontiguousarray(system.type, dtype=np.int32), device=device)
        b = np.ascontiguousarray(system.bonds, dtype=np.int32).reshape(-1, 2)
        self.nbond = b.shape[0]
        self.bonds = torch.as_tensor(b, device=device) if self.nbond else None
        self.r0 = torch.as_tensor(np.ascontiguousarray(system.r0), **f64) if self.nbond else None
        self.box = (C.c_double * 3)(*[float(v) for v in system.box])
        self.per = (C.c_int32 * 3)(*[int(v) for v in system.periodic])


def _step_times(h, enable):
    n = C.c_int64(0)
    gap = C.c_double(-1.0)
    _check(h, lib().rbc_step_times(h, int(bool(enable)), 0, None, C.byref(n), C.byref(gap)))
    ms = np.zeros(max(1, n.value))
    # the second call returns the same record (the timing switch is already set)
    _check(h, lib().rbc_step_times(h, int(bool(enable)), n.value, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(n), C.byref(gap)))
    return ms[:n.value], gap.value


def _host_times(h):
    host, wait = C.c_double(-1.0), C.c_double(-1.0)
    _check(h, lib().rbc_host_times(h, C.byref(host), C.byref(wait)))
    return host.value, wait.value


class Context:
    """One system on the current GPU (rbc_create / rbc_set_system / rbc_step ...)."""

    def __init__(self, mp, precision: int = RBC_FP64):
        self._h = C.c_void_p()
        self.params = make_params(mp, precision)
        _check(None, lib().rbc_create(C.byref(self.params), _stream_ptr(), C.byref(self._h)))
        self.n = 0

    def close(self):
        if self._h:
            lib().rbc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_system(self, system):
        u = _Uploaded(system)
        L = lib()
        _check(self._h, L.rbc_set_system(self._h, u.n, _dev(u.x), _dev(u.nrm), _dev(u.type), _dev(u.v), _dev(u.w),
                                         u.nbond, _dev(u.bonds), _dev(u.r0), u.box, u.per))
        self.n = u.n

    def update_cells(self, lloyd_iters: int = 0):
        _check(self._h, lib().rbc_update_cells(self._h, int(lloyd_iters)))

    def forces(self, energy: bool = False):
        import torch
        F = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        T = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        E = torch.zeros(2, dtype=torch.float64, device="cuda") if energy else None
        _check(self._h, lib().rbc_forces(self._h, _dev(F), _dev(T), _dev(E)))
        return (F, T, E) if energy else (F, T)

    def step(self, nsteps: int, dt: float):
        _check(self._h, lib().rbc_step(self._h, int(nsteps), float(dt)))

    def get_state(self):
        import torch
        out = [torch.empty((self.n, 3), dtype=torch.float64, device="cuda") for _ in range(4)]
        _check(self._h, lib().rbc_get_state(self._h, *[_dev(t) for t in out]))
        return out

    def get_pairs(self) -> np.ndarray:
        cnt = C.c_int64(0)
        _check(self._h, lib().rbc_get_pairs(self._h, 0, None, C.byref(cnt)))
        out = np.zeros((max(1, cnt.value), 2), dtype=np.int32)
        _check(self._h, lib().rbc_get_pairs(self._h, cnt.value, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                            C.byref(cnt)))
        return out[:cnt.value]

    def get_pairs_noalloc(self) -> np.ndarray:
        """As get_pairs, through the allocation-free export (rbc_get_pairs_noalloc)."""
        cnt = C.c_int64(0)
        _check(self._h, lib().rbc_get_pairs_noalloc(self._h, 0, None, C.byref(cnt)))
        out = np.zeros((max(1, cnt.value), 2), dtype=np.int32)
        _check(self._h, lib().rbc_get_pairs_noalloc(self._h, cnt.value, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                                    C.byref(cnt)))
        return out[:cnt.value]

    def energy(self) -> np.ndarray:
        out = np.zeros(7)
        _check(self._h, lib().rbc_energy(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def stats(self) -> dict:
        out = np.zeros(11, dtype=np.int64)
        _check(self._h, lib().rbc_stats(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))))
        keys = ["steps", "rebuilds", "early_rebuilds", "cells", "max_list_rows", "max_cell_pairs", "n", "lipids",
                "lipid_cells", "cell_updates", "prunes"]
        return dict(zip(keys, (int(v) for v in out)))

    def cells(self):
        st = self.stats()
        owner = np.zeros(self.n, dtype=np.int32)
        seeds = np.zeros((st["cells"], 3))
        _check(self._h, lib().rbc_get_cells(self._h, owner.ctypes.data_as(C.POINTER(C.c_int32)),
                                            seeds.ctypes.data_as(C.POINTER(C.c_double))))
        return owner, seeds

    def debug_array(self, which: int) -> np.ndarray:
        nb = C.c_int64(0)
        _check(self._h, lib().rbc_debug_array(self._h, int(which), 0, None, C.byref(nb)))
        dt = np.float64 if which == 7 else np.int32
        out = np.zeros(max(1, nb.value // np.dtype(dt).itemsize), dtype=dt)
        _check(self._h, lib().rbc_debug_array(self._h, int(which), nb.value, out.ctypes.data_as(C.c_void_p),
                                              C.byref(nb)))
        out = out[: nb.value // np.dtype(dt).itemsize]
        return out.reshape(-1, 4) if which == 7 else out

    def set_graphs(self, enable: bool = True):
        _check(self._h, lib().rbc_set_graphs(self._h, int(bool(enable))))

    def step_times(self, enable: bool = True):
        """As Ensemble.step_times."""
        return _step_times(self._h, enable)

    def host_times(self):
        """As Ensemble.host_times."""
        return _host_times(self._h)

    def force_timing(self, enable: bool = True):
        avg = C.c_double(0.0)
        cnt = C.c_int64(0)
        _check(self._h, lib().rbc_force_timing(self._h, int(enable), C.byref(avg), C.byref(cnt)))
        return avg.value, cnt.value

    def build_timing(self):
        """Average list-build kernel duration (ms) and launch count since the last call,
        timed while force timing is on."""
        avg = C.c_double(0.0)
        cnt = C.c_int64(0)
        _check(self._h, lib().rbc_build_timing(self._h, C.byref(avg), C.byref(cnt)))
        return avg.value, cnt.value

    def sync(self):
        _check(self._h, lib().rbc_sync(self._h))


class Ensemble:
    """Continuously batched systems (rbc_ensemble_*)."""

    def __init__(self, mp, precision: int = RBC_MIXED, max_slots: int = 64, hbm_budget: int = 0):
        self._h = C.c_void_p()
        self.params = make_params(mp, precision)
        _check(None, lib().rbc_ensemble_create(C.byref(self.params), _stream_ptr(), int(max_slots), int(hbm_budget),
                                               C.byref(self._h)))
        self.max_slots = int(max_slots)
        self.sizes = {}

    def close(self):
        if self._h:
            lib().rbc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, system) -> int:
        out = C.c_int64(0)
        nl = int(np.sum(system.type == 0))
        _check(self._h, lib().rbc_ensemble_footprint(self._h, system.N, nl, int(system.bonds.shape[0]),
                                                     C.byref(out)))
        return out.value

    def admit(self, system) -> Optional[int]:
        """Slot index, or None when no slot or budget is free.  A system that cannot be
        admitted at all (for example, its lists overflow the per-particle capacity)
        raises RbcError."""
        return self._admit(system, lib().rbc_ensemble_admit)

    def stage(self, system) -> Optional[int]:
        """As admit, with the cell build left to commit()."""
        return self._admit(system, lib().rbc_ensemble_stage)

    def commit(self) -> List[int]:
        """Build the cells of every staged system in one set of launches; returns the
        slots whose build failed (released; rbc_last_error names the first)."""
        failed = np.zeros(max(self.max_slots, 1), dtype=np.int32)
        nf = C.c_int64(0)
        _check(self._h, lib().rbc_ensemble_commit(self._h, failed.size, failed.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  C.byref(nf)))
        out = [int(q) for q in failed[:nf.value]]
        for q in out:
            self.sizes.pop(q, None)
        return out

    def _admit(self, system, fn) -> Optional[int]:
        u = _Uploaded(system)
        slot = C.c_int32(-1)
        st = fn(self._h, u.n, _dev(u.x), _dev(u.nrm), _dev(u.type), _dev(u.v), _dev(u.w),
                u.nbond, _dev(u.bonds), _dev(u.r0), u.box, u.per, C.byref(slot))
        if st == RBC_ERR_CAPACITY:
            info = self.info()
            if info["live"] >= self.max_slots or (
                    info["budget"] > 0 and info["bytes"] + self.footprint(system) > info["budget"]):
                return None
        _check(self._h, st)
        self.sizes[slot.value] = u.n
        return slot.value

    def step(self, nsteps: int, dt: float):
        _check(self._h, lib().rbc_ensemble_step(self._h, int(nsteps), float(dt)))

    def set_graphs(self, enable: bool = True):
        _check(self._h, lib().rbc_set_graphs(self._h, int(bool(enable))))

    def get_state(self, slot: int):
        import torch
        n = self.sizes.get(slot)
        if n is None:       # not a live slot here: the library reports it
            _check(self._h, lib().rbc_ensemble_get_state(self._h, int(slot), None, None, None, None))
            raise RbcError(RBC_ERR_NOT_READY, f"slot {slot} is not live")
        out = [torch.empty((n, 3), dtype=torch.float64, device="cuda") for _ in range(4)]
        _check(self._h, lib().rbc_ensemble_get_state(self._h, int(slot), *[_dev(t) for t in out]))
        return out

    def energy(self, slot: int) -> np.ndarray:
        out = np.zeros(7)
        _check(self._h, lib().rbc_ensemble_energy(self._h, int(slot), out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def retire(self, slot: int):
        _check(self._h, lib().rbc_ensemble_retire(self._h, int(slot)))
        self.sizes.pop(slot, None)

    def failed(self) -> dict:
        """Slots frozen by an error: {slot: status}."""
        n = C.c_int64(0)
        _check(self._h, lib().rbc_ensemble_failed(self._h, 0, None, None, C.byref(n)))
        slots = np.zeros(max(1, n.value), dtype=np.int32)
        st = np.zeros(max(1, n.value), dtype=np.int32)
        _check(self._h, lib().rbc_ensemble_failed(self._h, n.value, slots.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  st.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
        return {int(slots[q]): int(st[q]) for q in range(n.value)}

    def step_times(self, enable: bool = True):
        """Per-step GPU intervals (ms) of the last step call and the gap (ms) since the
        previous timed call (-1: none); turns step timing on or off for later calls."""
        return _step_times(self._h, enable)

    def host_times(self):
        """Microseconds per step of the last step call that the host spent deciding and
        launching, and waiting for earlier steps' drift statistics (-1 before any)."""
        return _host_times(self._h)

    def info(self) -> dict:
        out = np.zeros(4, dtype=np.int64)
        _check(self._h, lib().rbc_ensemble_info(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))))
        return dict(zip(["live", "bytes", "budget", "steps"], (int(v) for v in out)))
