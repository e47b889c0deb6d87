"""Initial structure generation from a triangular mesh (Initial structure generation
section of the paper), host side.

The mesh stands for the membrane at equilibrium shape; its triangles must be
oriented outward.  Following the paper's recipe:

* every vertex carries an actin junction and a glycophorin;
* every edge carries a spectrin chain and an immobile band-3;
* lipids and mobile band-3 are sampled uniformly on each triangle (the point
  (1 - sqrt r1) A + sqrt r1 (1 - r2) B + sqrt r1 r2 C of Osada et al., "Shape
  distributions", ACM TOG 2002, for uniform r1, r2), face by face in proportion
  to area, with a minimum distance between sampled particles and to the
  proteins in the sheet;
* the result is then relaxed by velocity quenching (rbc_params.quench) on the
  GPU before dynamics.

Readings (the paper gives the recipe, not the geometry or the types): the mesh
surface is the lipid sheet; actin sits ``depth`` under each vertex along the
vertex normal and the spectrin chains run between actin sites at that depth;
glycophorin sits on the vertex and immobile band-3 at the edge midpoint, each
bonded to the actin or the middle spectrin bead below it; mobile band-3 is free.
The model has three particle types: actin is the junction type, spectrin,
glycophorin and both band-3 kinds are protein beads (WCA with everything), and
their identities are returned separately.  Bond rest lengths equal the generated
distances, so the bonds start relaxed; the face sampling is what overlaps.
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np

from .inputs import LIPID, SPECTRIN, JUNCTION, LIPID_AREA, System

# identities of the generated particles (the model's types are coarser)
ACTIN, GLYCOPHORIN, SPECTRIN_BEAD, BAND3_IMMOBILE, BAND3_MOBILE, LIPID_ID = range(6)


@dataclasses.dataclass
class GenParams:
    lipid_area: float = LIPID_AREA     # sheet area per face-sampled particle (sigma^2)
    depth: float = 1.2                 # cytoskeleton depth under the sheet (sigma)
    beads_per_edge: int = 8            # spectrin beads on each edge
    band3_fraction: float = 0.01       # share of face-sampled particles that are mobile band-3
    min_dist: float = 0.7              # least distance of a face-sampled particle to the sheet's particles
    max_tries: int = 40                # redraw rounds before giving up on the remaining samples
    seed: int = 0


def mesh_edges(tri: np.ndarray) -> np.ndarray:
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=0)
    return np.unique(np.sort(e, axis=1), axis=0)


def face_normals_areas(v: np.ndarray, tri: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    a, b, c = (v[tri[:, k]] for k in range(3))
    cr = np.cross(b - a, c - a)
    nrm = np.linalg.norm(cr, axis=1)
    return cr / nrm[:, None], 0.5 * nrm


def vertex_normals(v: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Area-weighted mean of the incident face normals, normalised."""
    fn, fa = face_normals_areas(v, tri)
    acc = np.zeros_like(v)
    for k in range(3):
        np.add.at(acc, tri[:, k], fn * fa[:, None])
    return acc / np.linalg.norm(acc, axis=1)[:, None]


def sample_triangles(v: np.ndarray, tri: np.ndarray, faces: np.ndarray, rng) -> np.ndarray:
    """One uniform point on each listed face (Osada et al. 2002)."""
    r1 = np.sqrt(rng.random(faces.size))
    r2 = rng.random(faces.size)
    a, b, c = (v[tri[faces, k]] for k in range(3))
    return (1.0 - r1)[:, None] * a + (r1 * (1.0 - r2))[:, None] * b + (r1 * r2)[:, None] * c


def _accept_far(fixed: np.ndarray, cand: np.ndarray, dmin: float) -> np.ndarray:
    """Mask of candidates at least dmin from every fixed point and from every earlier
    accepted candidate (greedy in candidate order)."""
    from scipy.spatial import cKDTree
    ok = np.ones(cand.shape[0], dtype=bool)
    if fixed.shape[0]:
        d, _ = cKDTree(fixed).query(cand, k=1)
        ok &= d >= dmin
    idx = np.flatnonzero(ok)
    if idx.size > 1:
        pairs = cKDTree(cand[idx]).query_pairs(dmin, output_type="ndarray")
        if pairs.size:
            # greedy: walk the conflicts in order of their later member, dropping it if
            # its earlier partner is still kept
            pairs = pairs[np.lexsort((pairs[:, 0], pairs[:, 1]))]
            keep = np.ones(idx.size, dtype=bool)
            for i, j in pairs:
                if keep[i]:
                    keep[j] = False
            ok[idx[~keep]] = False
    return ok


def generate(vertices: np.ndarray, triangles: np.ndarray, gp: GenParams = GenParams(),
             name: str = "generated") -> Tuple[System, np.ndarray, np.ndarray]:
    """Build the two-component structure on the mesh.

    Returns (system, ident, face): ident[i] is the particle's identity (ACTIN ...
    LIPID_ID); face[i] the triangle a face-sampled particle was drawn on (-1 for
    the others).  Velocities are zero."""
    rng = np.random.default_rng(gp.seed)
    v = np.asarray(vertices, dtype=np.float64)
    tri = np.asarray(triangles, dtype=np.int64)
    nv = v.shape[0]
    edges = mesh_edges(tri)
    ne = edges.shape[0]
    vn = vertex_normals(v, tri)
    fn, fa = face_normals_areas(v, tri)
    m = int(gp.beads_per_edge)

    # vertices: glycophorin on the sheet, actin under it
    glyco = v.copy()
    actin = v - gp.depth * vn
    # edges: spectrin chain between the actin sites, immobile band-3 at the sheet midpoint
    k = np.arange(1, m + 1, dtype=np.float64) / (m + 1)
    a0, a1 = actin[edges[:, 0]], actin[edges[:, 1]]
    beads = (a0[:, None, :] + k[None, :, None] * (a1 - a0)[:, None, :]).reshape(ne * m, 3)
    band3 = 0.5 * (v[edges[:, 0]] + v[edges[:, 1]])

    # faces: lipids and mobile band-3, in proportion to area, at least min_dist from
    # the sheet's particles and from each other
    target = int(round(fa.sum() / gp.lipid_area))
    p_face = fa / fa.sum()
    sheet_fixed = np.concatenate([glyco, band3], axis=0)
    pts, pfaces = np.zeros((0, 3)), np.zeros(0, dtype=np.int64)
    for _ in range(gp.max_tries):
        need = target - pts.shape[0]
        if need <= 0:
            break
        faces = rng.choice(tri.shape[0], size=need, p=p_face)
        cand = sample_triangles(v, tri, faces, rng)
        ok = _accept_far(np.concatenate([sheet_fixed, pts], axis=0), cand, gp.min_dist)
        pts = np.concatenate([pts, cand[ok]], axis=0)
        pfaces = np.concatenate([pfaces, faces[ok]])
    nf = pts.shape[0]
    mobile = rng.random(nf) < gp.band3_fraction
    lip_pts, lip_faces = pts[~mobile], pfaces[~mobile]
    mob_pts, mob_faces = pts[mobile], pfaces[mobile]

    # assemble: lipids first (the model's convention), then proteins
    nL = lip_pts.shape[0]
    blocks = [(lip_pts, LIPID, LIPID_ID, lip_faces), (actin, JUNCTION, ACTIN, None),
              (glyco, SPECTRIN, GLYCOPHORIN, None), (beads, SPECTRIN, SPECTRIN_BEAD, None),
              (band3, SPECTRIN, BAND3_IMMOBILE, None), (mob_pts, SPECTRIN, BAND3_MOBILE, mob_faces)]
    x = np.concatenate([b[0] for b in blocks], axis=0)
    typ = np.concatenate([np.full(b[0].shape[0], b[1], dtype=np.int32) for b in blocks])
    ident = np.concatenate([np.full(b[0].shape[0], b[2], dtype=np.int32) for b in blocks])
    face = np.concatenate([b[3] if b[3] is not None else np.full(b[0].shape[0], -1, dtype=np.int64)
                           for b in blocks])
    off = np.cumsum([0] + [b[0].shape[0] for b in blocks])
    o_actin, o_glyco, o_beads, o_band3 = off[1], off[2], off[3], off[4]
    N = x.shape[0]
    nrm = np.zeros((N, 3))
    nrm[:nL] = fn[lip_faces]

    # bonds: actin - spectrin chain - actin, glycophorin - actin, band-3 - middle bead
    sid = o_beads + np.arange(ne * m).reshape(ne, m)
    chain = np.concatenate([(o_actin + edges[:, 0])[:, None], sid, (o_actin + edges[:, 1])[:, None]], axis=1)
    b_chain = np.stack([chain[:, :-1].ravel(), chain[:, 1:].ravel()], axis=1)
    b_glyco = np.stack([o_glyco + np.arange(nv), o_actin + np.arange(nv)], axis=1)
    b_band3 = np.stack([o_band3 + np.arange(ne), sid[:, m // 2]], axis=1)
    bonds = np.concatenate([b_chain, b_glyco, b_band3], axis=0).astype(np.int32)
    r0 = np.linalg.norm(x[bonds[:, 0]] - x[bonds[:, 1]], axis=1)

    system = System(name, x, nrm, typ, np.zeros((N, 3)), np.zeros((N, 3)), bonds, r0,
                    np.zeros(3), np.zeros(3, dtype=np.int32), 0.0)
    return system, ident, face
