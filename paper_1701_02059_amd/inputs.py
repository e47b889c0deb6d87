"""Seeded synthetic inputs for the two-component CGMD red-cell membrane model.

This module builds particle systems only: positions, orientations, types,
velocities and the bonded cytoskeleton topology, plus the model constants as
plain numbers.  It holds none of the force, neighbour-search, clustering or
integration arithmetic; both the FP64 CPU oracle and the HIP library consume
what it produces.

Geometry follows the paper's description of the whole-cell model (Initial
structure generation section; Introduction): lipid particles cover the
membrane surface one particle thick with outward orientations, and a
triangular spectrin network of junctions joined by bead chains sits just
under the sheet.  The paper gives no mesh file and no particle parameters,
so the constructions below are synthetic stand-ins with the paper's scale
(about 4 million particles for one cell, lipids about 80-90% of them).

Particle types: 0 = lipid (L), 1 = spectrin bead (S), 2 = junction (J).
IDs: lipids first in construction order, then junctions, then spectrin beads
edge by edge.  RNG: numpy PCG64 (``default_rng(seed)``) with the draw order
lipid jitter -> lipid tilt noise -> velocities -> angular velocities.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

LIPID, SPECTRIN, JUNCTION = 0, 1, 2
GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))
LIPID_AREA = 1.0911          # sigma^2 per lipid (hexagonal sheet at r_min)
ANCHOR_DEPTH = 1.2           # sigma, depth of the cytoskeleton under the sheet
DETACHED_DEPTH = 3.0         # sigma, depth of a detached cytoskeleton (beyond every lipid-protein cutoff)
DETACHED_TETHER = 2          # a detached cytoskeleton keeps the anchor bond of every 2nd junction
BEADS_PER_EDGE = 8


@dataclasses.dataclass
class ModelParams:
    """Model constants (sigma = epsilon = m = 1 units).

    The paper cites its membrane model without stating the potential or any
    constant; these values are a reading of the one-particle-thick
    orientation-dependent membrane potential that model builds on, WCA
    repulsion for protein beads and harmonic cytoskeleton bonds.
    """
    eps: float = 1.0
    zeta: float = 4.0
    mu: float = 3.0
    sin_theta0: float = 0.0
    r_min: float = 2.0 ** (1.0 / 6.0)
    r_c: float = 2.6
    wca_eps: float = 1.0
    wca_sigma: float = 1.0
    k_bond: float = 2.0
    mass: tuple = (1.0, 1.0, 1.0)
    inertia: float = 1.0
    cell_target: int = 16
    update_every: int = 100
    skin: float = 0.3
    inner_skin: float = 0.1       # pruned lists' buffer between list builds (see rbc_params.inner_skin)
    lloyd_iters: int = 10
    protein_cells: int = 0        # 1: protein beads get their own Voronoi cells (detached cytoskeleton)
    vol_k: float = 0.0            # harmonic volume constraint k_V (0: off)
    vol_target: float = 0.0       # V0; 0: the volume when the system is loaded
    lipid_area: float = LIPID_AREA
    kT: float = 0.22              # thermostat temperature
    gamma: float = 0.0            # Langevin friction rate on translations (0: off)
    gamma_rot: float = 0.0        # Langevin friction rate on lipid rotations (0: off)
    seed: int = 0                 # thermostat random stream
    quench: int = 0               # 1: velocity quenching (structure relaxation) instead of dynamics
    quench_max: float = 0.05      # largest move per quenching step (sigma; radians for rotations)

    def rc_table(self) -> np.ndarray:
        """Per type-pair cutoff: r_c for lipid-lipid, the WCA range otherwise."""
        t = np.full((3, 3), (2.0 ** (1.0 / 6.0)) * self.wca_sigma)
        t[LIPID, LIPID] = self.r_c
        return t


@dataclasses.dataclass
class System:
    name: str
    x: np.ndarray            # (N,3) f64 positions
    n: np.ndarray            # (N,3) f64 unit orientations (zero for proteins)
    type: np.ndarray         # (N,) int32
    v: np.ndarray            # (N,3) f64 velocities
    w: np.ndarray            # (N,3) f64 angular velocities (zero for proteins)
    bonds: np.ndarray        # (B,2) int32 particle ids
    r0: np.ndarray           # (B,) f64 rest lengths
    box: np.ndarray          # (3,) f64 box lengths (ignored on open axes)
    periodic: np.ndarray     # (3,) int32, 1 = periodic axis
    kT: float = 0.22

    @property
    def N(self) -> int:
        return int(self.x.shape[0])

    def counts(self) -> dict:
        return {"L": int(np.sum(self.type == LIPID)), "S": int(np.sum(self.type == SPECTRIN)),
                "J": int(np.sum(self.type == JUNCTION)), "bonds": int(self.bonds.shape[0])}

    def subset(self, idx: np.ndarray) -> "System":
        """Particles `idx` (ids renumbered in the given order), bonds inside the subset only."""
        idx = np.asarray(idx, dtype=np.int64)
        remap = -np.ones(self.N, dtype=np.int64)
        remap[idx] = np.arange(idx.size)
        keep = (remap[self.bonds[:, 0]] >= 0) & (remap[self.bonds[:, 1]] >= 0)
        b = remap[self.bonds[keep]].astype(np.int32)
        return System(self.name + "-subset", self.x[idx].copy(), self.n[idx].copy(),
                      self.type[idx].copy(), self.v[idx].copy(), self.w[idx].copy(),
                      b, self.r0[keep].copy(), self.box.copy(), self.periodic.copy(), self.kT)


# --------------------------------------------------------------------------- helpers

def _unit(a: np.ndarray) -> np.ndarray:
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def _fibonacci_sphere(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * GOLDEN_ANGLE
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def _hull_edges(points_on_sphere: np.ndarray) -> np.ndarray:
    from scipy.spatial import ConvexHull
    hull = ConvexHull(points_on_sphere)
    s = hull.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [2, 0]]], axis=0)
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int64)


def _velocities(rng, N: int, nL: int, n_lip: np.ndarray, kT: float, mass: np.ndarray, inertia: float):
    v = rng.normal(0.0, 1.0, size=(N, 3)) * np.sqrt(kT / mass)[:, None]
    vcm = (mass[:, None] * v).sum(axis=0) / mass.sum()
    v -= vcm
    g = rng.normal(0.0, math.sqrt(kT / inertia), size=(nL, 3))
    w_l = g - np.sum(g * n_lip, axis=1, keepdims=True) * n_lip
    w = np.zeros((N, 3))
    w[:nL] = w_l
    return v, w


def _chains(jpos: np.ndarray, edges: np.ndarray, nL: int, nJ: int, bead_pos_fn):
    """Beads along each edge plus the chain bonds (J-S-...-S-J, r0 = 1 sigma)."""
    nE = edges.shape[0]
    k = np.arange(1, BEADS_PER_EDGE + 1, dtype=np.float64) / (BEADS_PER_EDGE + 1)
    beads = bead_pos_fn(jpos[edges[:, 0]], jpos[edges[:, 1]], k)   # (nE, 8, 3)
    beads = beads.reshape(nE * BEADS_PER_EDGE, 3)
    s0 = nL + nJ
    sid = s0 + np.arange(nE * BEADS_PER_EDGE).reshape(nE, BEADS_PER_EDGE)
    ja = nL + edges[:, 0]
    jb = nL + edges[:, 1]
    chain = np.concatenate([ja[:, None], sid, jb[:, None]], axis=1)   # (nE, 10)
    bonds = np.stack([chain[:, :-1].ravel(), chain[:, 1:].ravel()], axis=1)
    return beads, bonds


def _anchor_bonds(jpos: np.ndarray, lip: np.ndarray, nL: int, box=None, periodic=None):
    from scipy.spatial import cKDTree
    if box is not None and periodic is not None and np.any(periodic):
        big = 1.0e6
        bs = np.where(periodic > 0, box, big)
        shift = np.where(periodic > 0, 0.0, big / 2)
        tree = cKDTree(np.mod(lip + shift, bs), boxsize=bs)
        _, idx = tree.query(np.mod(jpos + shift, bs))
    else:
        tree = cKDTree(lip)
        _, idx = tree.query(jpos)
    return np.stack([nL + np.arange(jpos.shape[0]), idx], axis=1)


def _assemble(name, lip, nrm, jpos, beads, chain_bonds, anchors, rng_state, kT, params, box, periodic,
              depth=ANCHOR_DEPTH):
    rng = rng_state
    nL, nJ, nS = lip.shape[0], jpos.shape[0], beads.shape[0]
    N = nL + nJ + nS
    x = np.concatenate([lip, jpos, beads], axis=0)
    n = np.zeros((N, 3))
    n[:nL] = nrm
    typ = np.concatenate([np.full(nL, LIPID), np.full(nJ, JUNCTION), np.full(nS, SPECTRIN)]).astype(np.int32)
    mass = np.asarray(params.mass, dtype=np.float64)[typ]
    v, w = _velocities(rng, N, nL, nrm, kT, mass, params.inertia)
    bonds = np.concatenate([chain_bonds, anchors], axis=0).astype(np.int32)
    r0 = np.concatenate([np.ones(chain_bonds.shape[0]), np.full(anchors.shape[0], depth)])
    return System(name, x, n, typ, v, w, bonds, r0, np.asarray(box, dtype=np.float64),
                  np.asarray(periodic, dtype=np.int32), kT)


# --------------------------------------------------------------------------- flat patch

def flat_patch(nx: int = 48, ny: int = 48, nj: int = 4, seed: int = 0, kT: float = 0.22,
               params: Optional[ModelParams] = None, spacing: float = 1.12,
               jitter: float = 0.02, tilt: float = 0.05, depth: float = ANCHOR_DEPTH,
               tether: int = 1) -> System:
    """Periodic flat bilayer patch on a triangular lattice (x, y periodic; z open).

    The cytoskeleton lies `depth` under the sheet; every `tether`-th junction keeps
    its anchor bond to the nearest lipid (1: all, an attached cytoskeleton)."""
    params = params or ModelParams()
    assert ny % 2 == 0 and nj % 2 == 0
    rng = np.random.default_rng(seed)
    Lx = nx * spacing
    Ly = ny * spacing * math.sqrt(3.0) / 2.0
    box = np.array([Lx, Ly, 0.0])
    periodic = np.array([1, 1, 0])
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel().astype(np.float64)
    j = j.ravel().astype(np.float64)
    lip = np.stack([(i + 0.5 * (j % 2)) * spacing, j * spacing * math.sqrt(3.0) / 2.0,
                    np.zeros_like(i)], axis=1)
    nL = lip.shape[0]
    lip = lip + rng.normal(0.0, jitter, size=(nL, 3))
    g = rng.normal(0.0, tilt, size=(nL, 2))
    nrm = _unit(np.stack([g[:, 0], g[:, 1], np.ones(nL)], axis=1))
    lip[:, :2] = np.mod(lip[:, :2], box[:2])
    # junction lattice
    ax, ay = Lx / nj, Ly / nj
    p, q = np.meshgrid(np.arange(nj), np.arange(nj), indexing="xy")
    p = p.ravel()
    q = q.ravel()
    jpos = np.stack([(p + 0.5 * (q % 2)) * ax, q * ay, np.full(p.shape, -depth)], axis=1).astype(np.float64)
    idx = lambda pp, qq: (qq % nj) * nj + (pp % nj)
    edges = []
    for a in range(nj * nj):
        pa, qa = a % nj, a // nj
        edges.append((a, idx(pa + 1, qa)))
        if qa % 2 == 0:
            edges.append((a, idx(pa - 1, qa + 1)))
            edges.append((a, idx(pa, qa + 1)))
        else:
            edges.append((a, idx(pa, qa + 1)))
            edges.append((a, idx(pa + 1, qa + 1)))
    edges = np.asarray(edges, dtype=np.int64)

    def beads_fn(a, b, k):
        d = b - a
        d[:, :2] -= np.rint(d[:, :2] / box[:2]) * box[:2]
        pts = a[:, None, :] + k[None, :, None] * d[:, None, :]
        pts[:, :, :2] = np.mod(pts[:, :, :2], box[:2])
        return pts

    beads, chain_bonds = _chains(jpos, edges, nL, jpos.shape[0], beads_fn)
    anchors = _anchor_bonds(jpos, lip, nL, box, periodic)[::tether]
    return _assemble(f"patch{nx}x{ny}", lip, nrm, jpos, beads, chain_bonds, anchors, rng, kT, params, box, periodic,
                     depth)


# --------------------------------------------------------------------------- vesicle

def vesicle(nL: int = 100_000, nJ: int = 1000, seed: int = 0, kT: float = 0.22,
            params: Optional[ModelParams] = None, jitter: float = 0.02, depth: float = ANCHOR_DEPTH,
            tether: int = 1) -> System:
    """Spherical vesicle: Fibonacci-sphere lipids, radial orientations, inner spectrin network
    `depth` under the sheet, anchored at every `tether`-th junction."""
    params = params or ModelParams()
    rng = np.random.default_rng(seed)
    R = math.sqrt(nL * 1.09 / (4.0 * math.pi))
    u = _fibonacci_sphere(nL)
    lip = R * u + rng.normal(0.0, jitter, size=(nL, 3))
    nrm = u.copy()
    uj = _fibonacci_sphere(nJ)
    Rj = R - depth
    jpos = Rj * uj
    edges = _hull_edges(uj)

    def beads_fn(a, b, k):
        ua, ub = _unit(a), _unit(b)
        om = np.arccos(np.clip(np.sum(ua * ub, axis=1), -1.0, 1.0))[:, None]
        so = np.sin(om)
        wa = np.sin((1.0 - k[None, :]) * om) / so
        wb = np.sin(k[None, :] * om) / so
        return Rj * (wa[:, :, None] * ua[:, None, :] + wb[:, :, None] * ub[:, None, :])

    beads, chain_bonds = _chains(jpos, edges, nL, nJ, beads_fn)
    anchors = _anchor_bonds(jpos, lip, nL)[::tether]
    return _assemble(f"vesicle{nL}", lip, nrm, jpos, beads, chain_bonds, anchors, rng, kT, params,
                     np.zeros(3), np.zeros(3, dtype=np.int32), depth)


# --------------------------------------------------------------------------- biconcave cell

EF_D_UM = 7.82
EF_C = (0.2072, 2.0026, -1.1228)


def evans_fung_meridian(t: np.ndarray, D: float = EF_D_UM, c=EF_C):
    """Evans-Fung biconcave meridian: rho(t) = R0 sin t, z(t) = (R0/2) cos t P(sin t), R0 = D/2.

    Returns rho, z, drho/dt, dz/dt.
    """
    R0 = D / 2.0
    c0, c1, c2 = c
    s, co = np.sin(t), np.cos(t)
    P = c0 + c1 * s ** 2 + c2 * s ** 4
    dP = 2.0 * c1 * s + 4.0 * c2 * s ** 3
    rho = R0 * s
    z = 0.5 * R0 * co * P
    drho = R0 * co
    dz = 0.5 * R0 * (-s * P + co * co * dP)
    return rho, z, drho, dz


def evans_fung_area_table(n: int = 400_001, D: float = EF_D_UM):
    t = np.linspace(0.0, math.pi, n)
    rho, z, drho, dz = evans_fung_meridian(t, D)
    f = 2.0 * math.pi * rho * np.sqrt(drho ** 2 + dz ** 2)
    A = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(t))])
    return t, A


def evans_fung_area_volume(n: int = 400_001, D: float = EF_D_UM):
    t, A = evans_fung_area_table(n, D)
    rho, z, drho, dz = evans_fung_meridian(t, D)
    g = -math.pi * rho ** 2 * dz
    V = float(np.sum(0.5 * (g[1:] + g[:-1]) * np.diff(t)))
    return float(A[-1]), V


def _ef_points(count: int, t_tab, A_tab, scale):
    Atot = A_tab[-1]
    i = np.arange(count, dtype=np.float64)
    target = (i + 0.5) / count * Atot
    t = np.interp(target, A_tab, t_tab)
    phi = i * GOLDEN_ANGLE
    rho, z, drho, dz = evans_fung_meridian(t)
    pos = scale * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    nm = np.stack([-dz * np.cos(phi), -dz * np.sin(phi), drho], axis=1)
    nm = _unit(nm)
    zs = 1.0 - 2.0 * np.interp(t, t_tab, A_tab) / Atot
    rs = np.sqrt(np.maximum(0.0, 1.0 - zs * zs))
    sph = np.stack([rs * np.cos(phi), rs * np.sin(phi), zs], axis=1)
    return pos, nm, sph


def biconcave_cell(nL: int = 3_600_000, nJ: int = 16_000, seed: int = 0, kT: float = 0.22,
                   params: Optional[ModelParams] = None, jitter: float = 0.02, depth: float = ANCHOR_DEPTH,
                   tether: int = 1) -> System:
    """Whole red cell: lipids by equal-area Fibonacci sampling of the Evans-Fung surface.

    The surface is scaled (sigma per micrometre) so that each lipid covers LIPID_AREA.
    Junctions use the same sampling, offset inward along the normal, triangulated
    through the equal-area map to the unit sphere.  Beads start at even fractions
    of the straight chord between their junctions and are then moved along the
    local surface normal (that of the nearest lipid site) to the same depth under
    the sheet as the junctions: on the strongly curved rim a bare chord would cut
    into the lipid layer.  Every `tether`-th junction keeps its anchor bond.
    """
    params = params or ModelParams()
    rng = np.random.default_rng(seed)
    t_tab, A_tab = evans_fung_area_table()
    scale = math.sqrt(nL * LIPID_AREA / A_tab[-1])
    site, nrm, _ = _ef_points(nL, t_tab, A_tab, scale)
    lip = site + rng.normal(0.0, jitter, size=(nL, 3))
    jp, jn, jsph = _ef_points(nJ, t_tab, A_tab, scale)
    jpos = jp - depth * jn
    edges = _hull_edges(jsph)

    def beads_fn(a, b, k):
        return a[:, None, :] + k[None, :, None] * (b - a)[:, None, :]

    beads, chain_bonds = _chains(jpos, edges, nL, nJ, beads_fn)
    beads = _to_depth(beads, site, nrm, depth)
    anchors = _anchor_bonds(jpos, lip, nL)[::tether]
    s = _assemble(f"rbc{nL + nJ + beads.shape[0]}", lip, nrm, jpos, beads, chain_bonds, anchors, rng, kT,
                  params, np.zeros(3), np.zeros(3, dtype=np.int32), depth)
    s.scale = scale
    return s


def _to_depth(p: np.ndarray, site: np.ndarray, nrm: np.ndarray, depth: float) -> np.ndarray:
    """Move points along the normal of their nearest surface site to `depth` below it."""
    from scipy.spatial import cKDTree
    _, idx = cKDTree(site).query(p)
    x0, n0 = site[idx], nrm[idx]
    h = np.sum((p - x0) * n0, axis=1)
    return p - (h + depth)[:, None] * n0


# --------------------------------------------------------------------------- triangular meshes

def _hull_triangles(points_on_sphere: np.ndarray) -> np.ndarray:
    """Triangles of the convex hull of points on the unit sphere, each ordered so that
    its normal (b - a) x (c - a) points away from the origin."""
    from scipy.spatial import ConvexHull
    tri = ConvexHull(points_on_sphere).simplices.astype(np.int64)
    a, b, c = (points_on_sphere[tri[:, k]] for k in range(3))
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def sphere_mesh(nv: int = 200, radius: float = 12.0):
    """Closed triangular mesh of a sphere: nv Fibonacci vertices, outward triangles."""
    u = _fibonacci_sphere(nv)
    return radius * u, _hull_triangles(u)


def evans_fung_mesh(nv: int = 2000, area: float = 450_000 * LIPID_AREA):
    """Closed triangular mesh of the Evans-Fung biconcave shape with nv equal-area
    vertices, scaled to the given surface area (sigma^2), triangulated through the
    equal-area map to the sphere; triangles oriented outward."""
    t_tab, A_tab = evans_fung_area_table()
    scale = math.sqrt(area / A_tab[-1])
    pos, _, sph = _ef_points(nv, t_tab, A_tab, scale)
    return pos, _hull_triangles(sph)


# --------------------------------------------------------------------------- named workloads

def patch_for_lipids(nL: int, seed: int, kT: float = 0.22, params=None) -> System:
    n = max(8, 2 * int(round(math.sqrt(nL) / 2.0)))
    nj = max(2, 2 * int(round(n / 12.0 / 2.0)))
    return flat_patch(n, n, nj, seed=seed, kT=kT, params=params)


def vesicle_for_lipids(nL: int, seed: int, kT: float = 0.22, params=None) -> System:
    return vesicle(nL, max(12, int(round(nL / 100.0))), seed=seed, kT=kT, params=params)


def config(name: str, seed: int = 0, params: Optional[ModelParams] = None) -> System:
    """The synthetic workloads: 'patch' (2,704 particles), 'vesicle' (124,952),
    'rbc4m' (3,999,952), 'rbc500k' (499,952), and 'tiny' for fast checks.  A
    '_detached' suffix gives the same sizes with the cytoskeleton DETACHED_DEPTH
    under the sheet and tethered at every DETACHED_TETHER-th junction only
    ('tiny_detached' is for static checks: on a sphere that small the deeper
    network crowds its chain beads at the junctions and does not hold together
    under dynamics)."""
    if name.endswith("_detached"):
        base = name[: -len("_detached")]
        kw = dict(seed=seed, params=params, depth=DETACHED_DEPTH, tether=DETACHED_TETHER)
        if base == "patch":
            return flat_patch(48, 48, 4, **kw)
        if base == "vesicle":
            return vesicle(100_000, 1000, **kw)
        if base == "rbc4m":
            return biconcave_cell(3_600_000, 16_000, **kw)
        if base == "rbc500k":
            return biconcave_cell(450_000, 2_000, **kw)
        if base == "tiny":
            return vesicle(2_000, 20, **kw)
        raise ValueError(name)
    if name == "patch":
        return flat_patch(48, 48, 4, seed=seed, params=params)
    if name == "vesicle":
        return vesicle(100_000, 1000, seed=seed, params=params)
    if name == "rbc4m":
        return biconcave_cell(3_600_000, 16_000, seed=seed, params=params)
    if name == "rbc500k":
        return biconcave_cell(450_000, 2_000, seed=seed, params=params)
    if name == "tiny":
        return vesicle(2_000, 20, seed=seed, params=params)
    raise ValueError(name)


def serving_requests(count: int = 256, rate: float = 20.0, seed: int = 12345,
                     lo: int = 2_000, hi: int = 200_000, steps: int = 500):
    """Request stream: Poisson arrivals; each a patch or a vesicle with log-uniform lipid count.

    Returns a list of dicts (arrival time, kind, lipid count, seed, steps); systems are
    built lazily with `build_request`.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.integers(0, 2, size=count)
    nl = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count)).astype(np.int64)
    return [{"id": r, "arrival": float(t[r]), "kind": "patch" if kinds[r] == 0 else "vesicle",
             "nL": int(nl[r]), "seed": r, "steps": steps} for r in range(count)]


def build_request(req: dict, params: Optional[ModelParams] = None) -> System:
    if req["kind"] == "patch":
        return patch_for_lipids(req["nL"], req["seed"], params=params)
    return vesicle_for_lipids(req["nL"], req["seed"], params=params)
