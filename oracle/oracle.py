"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
module.  The product path (the HIP library and its binding) never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rbc_oracle.c")
LIB = os.path.join(HERE, "librbc_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with every FP64 operation rounded separately (no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class OrcParams(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("periodic", C.c_int32 * 3), ("rc", (C.c_double * 3) * 3),
                ("eps", C.c_double), ("zeta", C.c_double), ("mu", C.c_double),
                ("sin_theta0", C.c_double), ("r_min", C.c_double),
                ("wca_eps", C.c_double), ("wca_sigma", C.c_double), ("k_bond", C.c_double),
                ("mass", C.c_double * 3), ("inertia", C.c_double)]


def make_params(mp, box=(0.0, 0.0, 0.0), periodic=(0, 0, 0)) -> OrcParams:
    p = OrcParams()
    for a in range(3):
        p.box[a] = float(box[a])
        p.periodic[a] = int(periodic[a])
    rc = mp.rc_table()
    for a in range(3):
        for b in range(3):
            p.rc[a][b] = float(rc[a, b])
    p.eps, p.zeta, p.mu, p.sin_theta0, p.r_min = mp.eps, mp.zeta, mp.mu, mp.sin_theta0, mp.r_min
    p.wca_eps, p.wca_sigma, p.k_bond = mp.wca_eps, mp.wca_sigma, mp.k_bond
    for a in range(3):
        p.mass[a] = float(mp.mass[a])
    p.inertia = mp.inertia
    return p


def params_for(system, mp) -> OrcParams:
    return make_params(mp, system.box, system.periodic)


class OrcExt(C.Structure):
    _fields_ = [("vol_k", C.c_double), ("vol_target", C.c_double), ("lipid_area", C.c_double),
                ("kT", C.c_double), ("gamma", C.c_double), ("gamma_rot", C.c_double), ("seed", C.c_uint64),
                ("quench_max", C.c_double), ("quench", C.c_int32), ("pad", C.c_int32)]


def make_ext(mp, vol_target=0.0) -> OrcExt:
    """Volume-constraint and thermostat constants of a ModelParams; V0 given explicitly."""
    e = OrcExt()
    e.vol_k, e.vol_target, e.lipid_area = float(mp.vol_k), float(vol_target), float(mp.lipid_area)
    e.kT, e.gamma, e.gamma_rot, e.seed = float(mp.kT), float(mp.gamma), float(mp.gamma_rot), int(mp.seed)
    e.quench, e.quench_max = int(mp.quench), float(mp.quench_max)
    return e


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        P = C.POINTER
        dp, ip, i64p, u64p = P(C.c_double), P(C.c_int32), P(C.c_int64), P(C.c_uint64)
        pp = P(OrcParams)
        ep = P(OrcExt)
        sig = {
            "orc_dist2": (C.c_double, [pp, dp, dp, dp]),
            "orc_pair_lipid": (C.c_double, [pp, dp, dp, dp, dp, dp, dp]),
            "orc_pair_wca": (C.c_double, [pp, dp, dp]),
            "orc_bond": (C.c_double, [pp, dp, C.c_double, dp]),
            "orc_pairs_brute": (C.c_int64, [pp, C.c_int64, dp, ip, C.c_int64, ip]),
            "orc_pairs_grid": (C.c_int64, [pp, C.c_int64, dp, ip, C.c_int64, ip]),
            "orc_forces": (C.c_int, [pp, C.c_int64, dp, dp, ip, C.c_int64, ip, dp, dp, dp, dp, C.c_int]),
            "orc_forces_subset": (C.c_int, [pp, C.c_int64, dp, dp, ip, C.c_int64, ip, dp, C.c_int64, i64p,
                                            dp, dp, C.c_int]),
            "orc_assign": (None, [pp, C.c_int64, dp, C.c_int64, dp, ip]),
            "orc_seed_update": (None, [pp, C.c_int64, dp, ip, ip, C.c_int64, dp]),
            "orc_morton": (None, [pp, C.c_int64, dp, u64p]),
            "orc_cell_bounds": (None, [pp, C.c_int64, dp, ip, C.c_int64, dp, dp]),
            "orc_cell_pairs": (C.c_int64, [pp, C.c_int64, dp, dp, C.c_double, C.c_double, C.c_int64, ip]),
            "orc_vv_run": (C.c_int, [pp, C.c_int64, dp, dp, dp, dp, ip, C.c_int64, ip, dp, C.c_double,
                                     C.c_int64, dp, C.c_int]),
            "orc_philox4x32_10": (None, [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]),
            "orc_volume": (C.c_double, [ep, C.c_int64, dp, dp, ip]),
            "orc_volume_forces": (C.c_double, [ep, C.c_int64, dp, dp, ip, dp, dp]),
            "orc_forces_ext": (C.c_int, [pp, ep, C.c_int64, dp, dp, ip, C.c_int64, ip, dp, dp, dp, dp, C.c_int]),
            "orc_langevin_step": (None, [pp, ep, C.c_int64, ip, dp, C.c_double, C.c_uint64, dp, dp]),
            "orc_quench_project": (None, [pp, C.c_int64, ip, dp, dp, dp, dp]),
            "orc_quench_cap": (None, [ep, C.c_int64, ip, C.c_double, dp, dp]),
            "orc_vv_run_ext": (C.c_int, [pp, ep, C.c_uint64, C.c_int64, dp, dp, dp, dp, ip, C.c_int64, ip, dp,
                                         C.c_double, C.c_int64, dp, C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def dist2(p, xi, xj):
    d = np.zeros(3)
    _, pi_ = _d(xi)
    _, pj_ = _d(xj)
    r = lib().orc_dist2(C.byref(p), pi_, pj_, d.ctypes.data_as(C.POINTER(C.c_double)))
    return r, d


def pair_lipid(p, d, ni, nj):
    Fi, ti, tj = np.zeros(3), np.zeros(3), np.zeros(3)
    dd, ni_, nj_ = _d(d), _d(ni), _d(nj)
    U = lib().orc_pair_lipid(C.byref(p), dd[1], ni_[1], nj_[1], _d(Fi)[1], _d(ti)[1], _d(tj)[1])
    return U, Fi, ti, tj


def pair_wca(p, d):
    Fi = np.zeros(3)
    U = lib().orc_pair_wca(C.byref(p), _d(d)[1], _d(Fi)[1])
    return U, Fi


def bond(p, d, r0):
    Fi = np.zeros(3)
    U = lib().orc_bond(C.byref(p), _d(d)[1], float(r0), _d(Fi)[1])
    return U, Fi


def pairs(p, x, typ, method="grid"):
    x, xp = _d(x)
    typ, tp = _i(typ)
    n = x.shape[0]
    f = lib().orc_pairs_grid if method == "grid" else lib().orc_pairs_brute
    cap = max(1024, 40 * n)
    while True:
        out = np.zeros((cap, 2), dtype=np.int32)
        cnt = f(C.byref(p), n, xp, tp, cap, out.ctypes.data_as(C.POINTER(C.c_int32)))
        if cnt <= cap:
            return out[:cnt].copy()
        cap = int(cnt)


def forces(p, system, x=None, nrm=None, nthreads=0):
    x = system.x if x is None else x
    nrm = system.n if nrm is None else nrm
    x, xp = _d(x)
    nrm, np_ = _d(nrm)
    typ, tp = _i(system.type)
    b, bp = _i(system.bonds.reshape(-1, 2))
    r0, r0p = _d(system.r0)
    n = x.shape[0]
    F, T, en = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(2)
    lib().orc_forces(C.byref(p), n, xp, np_, tp, b.shape[0], bp, r0p, _d(F)[1], _d(T)[1], _d(en)[1], nthreads)
    return F, T, en[0], en[1]


def forces_subset(p, system, idx, x=None, nrm=None, nthreads=0):
    x = system.x if x is None else x
    nrm = system.n if nrm is None else nrm
    x, xp = _d(x)
    nrm, np_ = _d(nrm)
    typ, tp = _i(system.type)
    b, bp = _i(system.bonds.reshape(-1, 2))
    r0, r0p = _d(system.r0)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    F, T = np.zeros((idx.size, 3)), np.zeros((idx.size, 3))
    lib().orc_forces_subset(C.byref(p), x.shape[0], xp, np_, tp, b.shape[0], bp, r0p, idx.size,
                            idx.ctypes.data_as(C.POINTER(C.c_int64)), _d(F)[1], _d(T)[1], nthreads)
    return F, T


def assign(p, x, seeds):
    x, xp = _d(x)
    s, sp = _d(seeds)
    owner = np.zeros(x.shape[0], dtype=np.int32)
    lib().orc_assign(C.byref(p), x.shape[0], xp, s.shape[0], sp, owner.ctypes.data_as(C.POINTER(C.c_int32)))
    return owner


def seed_update(p, x, typ, owner, seeds):
    x, xp = _d(x)
    typ, tp = _i(typ)
    owner, op = _i(owner)
    s = np.array(seeds, dtype=np.float64, copy=True)
    lib().orc_seed_update(C.byref(p), x.shape[0], xp, tp, op, s.shape[0], s.ctypes.data_as(C.POINTER(C.c_double)))
    return s


def morton(p, seeds):
    s, sp = _d(seeds)
    keys = np.zeros(s.shape[0], dtype=np.uint64)
    lib().orc_morton(C.byref(p), s.shape[0], sp, keys.ctypes.data_as(C.POINTER(C.c_uint64)))
    return keys


def cell_bounds(p, x, owner, seeds):
    x, xp = _d(x)
    owner, op = _i(owner)
    s, sp = _d(seeds)
    R = np.zeros(s.shape[0])
    lib().orc_cell_bounds(C.byref(p), x.shape[0], xp, op, s.shape[0], sp, R.ctypes.data_as(C.POINTER(C.c_double)))
    return R


def cell_pairs(p, seeds, R, rs, skin):
    s, sp = _d(seeds)
    R, rp = _d(R)
    k = s.shape[0]
    cap = max(1024, 64 * k)
    while True:
        out = np.zeros((cap, 2), dtype=np.int32)
        cnt = lib().orc_cell_pairs(C.byref(p), k, sp, rp, float(rs), float(skin), cap,
                                   out.ctypes.data_as(C.POINTER(C.c_int32)))
        if cnt <= cap:
            return out[:cnt].copy()
        cap = int(cnt)


def vv_run(p, system, dt, nsteps, nthreads=0):
    """Run NVE velocity Verlet on copies of the system state; returns (x, v, n, w, energies)."""
    x = np.array(system.x, dtype=np.float64, copy=True)
    v = np.array(system.v, dtype=np.float64, copy=True)
    nrm = np.array(system.n, dtype=np.float64, copy=True)
    w = np.array(system.w, dtype=np.float64, copy=True)
    typ, tp = _i(system.type)
    b, bp = _i(system.bonds.reshape(-1, 2))
    r0, r0p = _d(system.r0)
    en = np.zeros((nsteps + 1, 3))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    lib().orc_vv_run(C.byref(p), x.shape[0], dp(x), dp(v), dp(nrm), dp(w), tp, b.shape[0], bp, r0p,
                     float(dt), int(nsteps), dp(en), nthreads)
    return x, v, nrm, w, en


# ---------------------------------------------------------------- Voronoi reference pipeline

def voronoi_init(p, system, m, lloyd_iters):
    """Initial seeds: lipid number floor(j*N_L/k), then Lloyd iterations (E then M)."""
    lip = np.flatnonzero(system.type == 0)
    nL = lip.size
    k = -(-nL // m)
    seeds = system.x[lip[(np.arange(k) * nL) // k]].copy()
    for a in range(3):
        if system.periodic[a]:
            seeds[:, a] = seeds[:, a] - system.box[a] * np.floor(seeds[:, a] / system.box[a])
    owner = None
    for _ in range(lloyd_iters):
        owner = assign(p, system.x, seeds)
        seeds = seed_update(p, system.x, system.type, owner, seeds)
    return seeds, owner


def voronoi_update(p, x, typ, seeds, owner_prev_order=None):
    """One online-EM update: E, M, Morton sort of seeds and renumbering, stable particle order.

    Returns (new_seeds, new_owner, order) where order is the stable sort of particles
    (in the given order) by their new owner.
    """
    owner = assign(p, x, seeds)
    seeds = seed_update(p, x, typ, owner, seeds)
    keys = morton(p, seeds)
    perm = np.lexsort((np.arange(keys.size), keys))      # by key, then previous index
    new_index = np.empty_like(perm)
    new_index[perm] = np.arange(perm.size)
    seeds = seeds[perm]
    owner = new_index[owner].astype(np.int32)
    order = np.argsort(owner, kind="stable")
    return seeds, owner, order


# ------------------------------------------- two cell sets (detached cytoskeleton)
# Force Evaluation section: for a cytoskeleton that has left the bilayer, the
# protein beads get a Voronoi cell set of their own, built like the lipids' one.
# Cells [0, kl) are the lipids' and [kl, k) the proteins'; every step above runs
# within each set, and the Morton renumbering keeps the lipid cells first.

def set_sizes(typ, m):
    """(kl, kp): ceil(N_L / m) lipid cells and ceil(N_P / m) protein cells."""
    nL = int(np.count_nonzero(np.asarray(typ) == 0))
    nP = int(np.asarray(typ).size) - nL
    return -(-nL // m), -(-nP // m)


def assign_sets(p, x, typ, seeds, kl):
    """E-step per set: a lipid's nearest lipid cell, a protein bead's nearest protein cell."""
    lip = np.asarray(typ) == 0
    owner = np.empty(x.shape[0], dtype=np.int32)
    owner[lip] = assign(p, x[lip], seeds[:kl])
    owner[~lip] = assign(p, x[~lip], seeds[kl:]) + kl
    return owner


def seed_update_sets(p, x, typ, owner, seeds, kl):
    """M-step per set: lipid cells move to the mean of their lipid members,
    protein cells to the mean of their protein members."""
    lip = np.asarray(typ) == 0
    out = np.array(seeds, dtype=np.float64, copy=True)
    out[:kl] = seed_update(p, x[lip], np.asarray(typ)[lip], owner[lip], seeds[:kl])
    # within the protein set every member counts: present them as the averaged kind
    nP = int(np.count_nonzero(~lip))
    out[kl:] = seed_update(p, x[~lip], np.zeros(nP, dtype=np.int32), owner[~lip] - kl, seeds[kl:])
    return out


def morton_sets(p, seeds, kl):
    """Morton keys over all centroids, with bit 63 set on the protein set's cells."""
    keys = morton(p, seeds)
    keys[kl:] |= np.uint64(1) << np.uint64(63)
    return keys


def voronoi_init_sets(p, system, m, lloyd_iters):
    """Initial seeds of both sets (lipid number floor(j*N_L/kl), protein number
    floor(j*N_P/kp)), then Lloyd iterations within each set.  Returns (seeds, owner, kl)."""
    typ = np.asarray(system.type)
    lip = np.flatnonzero(typ == 0)
    prot = np.flatnonzero(typ != 0)
    kl, kp = set_sizes(typ, m)
    seeds = np.concatenate([system.x[lip[(np.arange(kl) * lip.size) // kl]],
                            system.x[prot[(np.arange(kp) * prot.size) // max(kp, 1)]][:kp]])
    for a in range(3):
        if system.periodic[a]:
            seeds[:, a] = seeds[:, a] - system.box[a] * np.floor(seeds[:, a] / system.box[a])
    owner = None
    for _ in range(lloyd_iters):
        owner = assign_sets(p, system.x, typ, seeds, kl)
        seeds = seed_update_sets(p, system.x, typ, owner, seeds, kl)
    return seeds, owner, kl


def voronoi_update_sets(p, x, typ, seeds, kl):
    """One online-EM update with two cell sets (as voronoi_update); returns
    (new_seeds, new_owner, order)."""
    owner = assign_sets(p, x, typ, seeds, kl)
    seeds = seed_update_sets(p, x, typ, owner, seeds, kl)
    keys = morton_sets(p, seeds, kl)
    perm = np.lexsort((np.arange(keys.size), keys))
    new_index = np.empty_like(perm)
    new_index[perm] = np.arange(perm.size)
    seeds = seeds[perm]
    owner = new_index[owner].astype(np.int32)
    order = np.argsort(owner, kind="stable")
    return seeds, owner, order


# ------------------------------------------- volume constraint and thermostat

def philox(ctr, key):
    """Philox4x32-10 of a 4-word counter and 2-word key."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    out = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def volume(e, x, nrm, typ):
    x, xp = _d(x)
    nrm, np_ = _d(nrm)
    typ, tp = _i(typ)
    return float(lib().orc_volume(C.byref(e), x.shape[0], xp, np_, tp))


def volume_forces(e, x, nrm, typ):
    """(F, T, U_V) of the volume term alone."""
    x, xp = _d(x)
    nrm, np_ = _d(nrm)
    typ, tp = _i(typ)
    F, T = np.zeros_like(x), np.zeros_like(x)
    U = lib().orc_volume_forces(C.byref(e), x.shape[0], xp, np_, tp, _d(F)[1], _d(T)[1])
    return F, T, float(U)


def forces_ext(p, e, system, x=None, nrm=None, nthreads=0):
    x = system.x if x is None else x
    nrm = system.n if nrm is None else nrm
    x, xp = _d(x)
    nrm, np_ = _d(nrm)
    typ, tp = _i(system.type)
    b, bp = _i(system.bonds.reshape(-1, 2))
    r0, r0p = _d(system.r0)
    n = x.shape[0]
    F, T, en = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(2)
    lib().orc_forces_ext(C.byref(p), C.byref(e), n, xp, np_, tp, b.shape[0], bp, r0p, _d(F)[1], _d(T)[1],
                         _d(en)[1], nthreads)
    return F, T, en[0], en[1]


def langevin_step(p, e, typ, nrm, dt, step, v, w):
    """The thermostat update on copies of v and w; returns (v, w)."""
    typ, tp = _i(typ)
    nrm, np_ = _d(nrm)
    v = np.array(v, dtype=np.float64, copy=True)
    w = np.array(w, dtype=np.float64, copy=True)
    lib().orc_langevin_step(C.byref(p), C.byref(e), typ.shape[0], tp, np_, float(dt), int(step),
                            _d(v)[1], _d(w)[1])
    return v, w


def vv_run_ext(p, e, system, dt, nsteps, step0=0, nthreads=0):
    """Velocity Verlet with the volume term and the thermostat on copies of the state;
    returns (x, v, n, w, energies)."""
    x = np.array(system.x, dtype=np.float64, copy=True)
    v = np.array(system.v, dtype=np.float64, copy=True)
    nrm = np.array(system.n, dtype=np.float64, copy=True)
    w = np.array(system.w, dtype=np.float64, copy=True)
    typ, tp = _i(system.type)
    b, bp = _i(system.bonds.reshape(-1, 2))
    r0, r0p = _d(system.r0)
    en = np.zeros((nsteps + 1, 3))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    lib().orc_vv_run_ext(C.byref(p), C.byref(e), int(step0), x.shape[0], dp(x), dp(v), dp(nrm), dp(w), tp,
                         b.shape[0], bp, r0p, float(dt), int(nsteps), dp(en), nthreads)
    return x, v, nrm, w, en


def quench_project(p, typ, F, T, v, w):
    """The quench projection on copies of v and w; returns (v, w)."""
    typ, tp = _i(typ)
    F, Fp = _d(F)
    T, Tp = _d(T)
    v = np.array(v, dtype=np.float64, copy=True)
    w = np.array(w, dtype=np.float64, copy=True)
    lib().orc_quench_project(C.byref(p), typ.shape[0], tp, Fp, Tp, _d(v)[1], _d(w)[1])
    return v, w


def quench_cap(e, typ, dt, v, w):
    typ, tp = _i(typ)
    v = np.array(v, dtype=np.float64, copy=True)
    w = np.array(w, dtype=np.float64, copy=True)
    lib().orc_quench_cap(C.byref(e), typ.shape[0], tp, float(dt), _d(v)[1], _d(w)[1])
    return v, w
