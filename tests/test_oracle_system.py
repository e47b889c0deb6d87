"""Oracle pins at system level: neighbour set, force totals, Voronoi reference
steps and the velocity-Verlet / linear-rotor integrator."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_02059_amd import inputs as I


@pytest.fixture(scope="module")
def patch():
    return I.config("patch")


@pytest.fixture(scope="module")
def ves():
    return I.config("vesicle")


# ------------------------------------------------------------------ neighbour set

def test_patch_pair_set_brute_equals_grid_and_lattice_count(patch, mp):
    p = O.params_for(patch, mp)
    pb = O.pairs(p, patch.x, patch.type, "brute")
    pg = O.pairs(p, patch.x, patch.type, "grid")
    assert np.array_equal(pb, pg)
    ll = (patch.type[pb[:, 0]] == 0) & (patch.type[pb[:, 1]] == 0)
    assert int(ll.sum()) == 20736          # 18 lattice neighbours within 2.6 sigma per lipid
    deg = np.bincount(pb[ll].ravel(), minlength=2304)[:2304]
    assert np.all(deg == 18)


@pytest.mark.parametrize("size,seed", [(2000, 0), (8000, 1), (20000, 2)])
def test_vesicle_subsets_brute_equals_grid(ves, mp, size, seed):
    rng = np.random.default_rng(seed)
    # a contiguous cap of the vesicle plus random extra particles: dense and sparse regions
    c = ves.x[rng.integers(ves.N)]
    order = np.argsort(np.linalg.norm(ves.x - c, axis=1))
    idx = np.concatenate([order[: size // 2], rng.choice(ves.N, size // 2, replace=False)])
    idx = np.unique(idx)
    sub = ves.subset(idx)
    p = O.params_for(sub, mp)
    assert np.array_equal(O.pairs(p, sub.x, sub.type, "brute"), O.pairs(p, sub.x, sub.type, "grid"))


def test_grid_handles_small_periodic_box(mp):
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 6.0, size=(300, 3))
    typ = rng.integers(0, 3, size=300).astype(np.int32)
    p = O.make_params(mp, box=(6.0, 6.0, 0.0), periodic=(1, 1, 0))
    assert np.array_equal(O.pairs(p, x, typ, "brute"), O.pairs(p, x, typ, "grid"))


# ------------------------------------------------------------------ totals

def test_force_totals_patch(patch, mp):
    p = O.params_for(patch, mp)
    F, T, U, W = O.forces(p, patch)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale
    # energy equals the sum of pair energies plus bond energies (definition), written out here
    pairs = O.pairs(p, patch.x, patch.type, "brute")
    Usum = 0.0
    for i, j in pairs:
        _, d = O.dist2(p, patch.x[i], patch.x[j])
        if patch.type[i] == 0 and patch.type[j] == 0:
            Usum += O.pair_lipid(p, d, patch.n[i], patch.n[j])[0]
        else:
            Usum += O.pair_wca(p, d)[0]
    for (a, b), r0 in zip(patch.bonds, patch.r0):
        _, d = O.dist2(p, patch.x[a], patch.x[b])
        Usum += O.bond(p, d, r0)[0]
    assert U == pytest.approx(Usum, rel=1e-12)


def test_force_totals_vesicle_open_boundaries(ves, mp):
    p = O.params_for(ves, mp)
    F, T, U, W = O.forces(p, ves)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale
    L = np.cross(ves.x, F).sum(axis=0) + T.sum(axis=0)
    assert np.abs(L).max() < 1e-12 * (np.abs(np.cross(ves.x, F)).sum())
    # torques only on lipids and perpendicular to their orientation
    assert not T[ves.type != 0].any()
    lip = ves.type == 0
    assert np.abs(np.sum(T[lip] * ves.n[lip], axis=1)).max() < 1e-10


def test_total_energy_finite_difference(patch, mp):
    p = O.params_for(patch, mp)
    F, T, U, W = O.forces(p, patch)
    rng = np.random.default_rng(8)
    h = 1e-6
    for i in list(rng.choice(2304, 4, replace=False)) + [2304, 2320]:   # lipids, a junction, a bead
        for a in range(3):
            xp = patch.x.copy(); xp[i, a] += h
            xm = patch.x.copy(); xm[i, a] -= h
            Up = O.forces(p, patch, x=xp)[2]
            Um = O.forces(p, patch, x=xm)[2]
            assert F[i, a] == pytest.approx(-(Up - Um) / (2 * h), abs=2e-5 * max(1, abs(F[i, a])))


def test_subset_forces_equal_full(ves, mp):
    p = O.params_for(ves, mp)
    sub = ves.subset(np.arange(0, ves.N, 25))
    ps = O.params_for(sub, mp)
    F, T, _, _ = O.forces(ps, sub)
    idx = np.arange(0, sub.N, 37)
    Fs, Ts = O.forces_subset(ps, sub, idx)
    assert np.allclose(Fs, F[idx], rtol=0, atol=1e-12 * max(1.0, np.abs(F).max()))
    assert np.allclose(Ts, T[idx], rtol=0, atol=1e-12 * max(1.0, np.abs(T).max()))


def test_virial_is_pair_sum(patch, mp):
    # W = sum over pairs of r_ij . F_ij (pairs and bonds), computed term by term
    p = O.params_for(patch, mp)
    _, _, _, W = O.forces(p, patch)
    pairs = O.pairs(p, patch.x, patch.type, "brute")
    Wsum = 0.0
    for i, j in pairs:
        _, d = O.dist2(p, patch.x[i], patch.x[j])
        if patch.type[i] == 0 and patch.type[j] == 0:
            Fi = O.pair_lipid(p, d, patch.n[i], patch.n[j])[1]
        else:
            Fi = O.pair_wca(p, d)[1]
        Wsum += d @ Fi
    for (a, b), r0 in zip(patch.bonds, patch.r0):
        _, d = O.dist2(p, patch.x[a], patch.x[b])
        Wsum += d @ O.bond(p, d, r0)[1]
    assert W == pytest.approx(Wsum, rel=1e-12)


# ------------------------------------------------------------------ Voronoi reference

def test_assign_matches_kdtree(mp):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(9)
    x = rng.normal(size=(5000, 3)) * 20
    seeds = rng.normal(size=(300, 3)) * 20
    p = O.make_params(mp)
    own = O.assign(p, x, seeds)
    _, ref = cKDTree(seeds).query(x)
    assert np.array_equal(own, ref)


def test_assign_ties_go_to_lowest_index(mp):
    p = O.make_params(mp)
    seeds = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0]])
    own = O.assign(p, np.array([[0.0, 0, 0], [0.0, 0.0, 5.0]]), seeds)
    assert list(own) == [0, 0]


def test_assign_periodic_min_image(mp):
    p = O.make_params(mp, box=(10.0, 10.0, 0.0), periodic=(1, 1, 0))
    seeds = np.array([[0.5, 5.0, 0.0], [7.0, 5.0, 0.0]])
    own = O.assign(p, np.array([[9.9, 5.0, 0.0]]), seeds)   # 0.6 away through the boundary
    assert own[0] == 0


def test_seed_update_is_lipid_centroid_and_lloyd_decreases(ves, mp):
    p = O.params_for(ves, mp)
    seeds, owner = O.voronoi_init(p, ves, 16, 1)
    lip = ves.type == 0
    obj = []
    for _ in range(5):
        owner = O.assign(p, ves.x, seeds)
        d = ves.x[lip] - seeds[owner[lip]]
        obj.append(float((d * d).sum()))
        new = O.seed_update(p, ves.x, ves.type, owner, seeds)
        # centroid of the lipid members (plain numpy)
        for s in (0, 17, 123):
            m = lip & (owner == s)
            if m.any():
                assert np.allclose(new[s], ves.x[m].mean(axis=0), atol=1e-10)
        seeds = new
    assert all(b <= a * (1 + 1e-12) for a, b in zip(obj, obj[1:]))


def test_seed_update_empty_and_protein_only_cells_stay(mp):
    p = O.make_params(mp)
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [5.0, 5, 5]])
    typ = np.array([0, 0, 1], dtype=np.int32)
    seeds = np.array([[0.2, 0, 0], [5.1, 5, 5], [9.0, 9, 9]])
    owner = np.array([0, 0, 1], dtype=np.int32)
    new = O.seed_update(p, x, typ, owner, seeds)
    assert np.allclose(new[0], [0.5, 0, 0])
    assert np.array_equal(new[1], seeds[1]) and np.array_equal(new[2], seeds[2])


def test_seed_update_periodic_wraps(mp):
    p = O.make_params(mp, box=(10.0, 10.0, 0.0), periodic=(1, 1, 0))
    x = np.array([[9.8, 1.0, 0.0], [0.4, 1.0, 0.0]])
    new = O.seed_update(p, x, np.zeros(2, np.int32), np.zeros(2, np.int32), np.array([[9.9, 1.0, 0.0]]))
    assert new[0] == pytest.approx([0.1, 1.0, 0.0])


def test_morton_hand_computed(mp):
    p = O.make_params(mp)
    seeds = np.array([[0.0, 0, 0], [1.0, 1, 1], [1.0, 0, 0], [0.0, 0, 1.0], [0.5, 0, 0]])
    k = O.morton(p, seeds)
    xbits = sum(1 << (3 * b + 2) for b in range(21))
    zbits = sum(1 << (3 * b) for b in range(21))
    assert k[0] == 0
    assert k[1] == (1 << 63) - 1
    assert k[2] == xbits
    assert k[3] == zbits
    assert k[4] == 1 << (3 * 20 + 2)           # x = half the extent -> top x bit only


def test_cell_pairs_cover_every_neighbour_pair(ves, mp):
    sub = ves.subset(np.arange(0, 30000))
    p = O.params_for(sub, mp)
    seeds, owner = O.voronoi_init(p, sub, 16, 3)
    R = O.cell_bounds(p, sub.x, owner, seeds)
    for s in range(0, seeds.shape[0], 97):
        m = owner == s
        if m.any():
            assert R[s] >= np.linalg.norm(sub.x[m] - seeds[s], axis=1).max() - 1e-12
    cp = O.cell_pairs(p, seeds, R, 2.6, 0.0)
    cset = set(map(tuple, cp))
    pairs = O.pairs(p, sub.x, sub.type)
    a, b = owner[pairs[:, 0]], owner[pairs[:, 1]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    assert all((int(u), int(v)) in cset for u, v in zip(lo, hi))


# ------------------------------------------- two cell sets (detached cytoskeleton)

def _two_set_cloud(seed=21, nl=400, npr=90):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(size=(nl, 3)) * 6, rng.normal(size=(npr, 3)) * 6 + [0, 0, 2.0]])
    typ = np.concatenate([np.zeros(nl), rng.integers(1, 3, npr)]).astype(np.int32)
    return x, typ


def test_assign_sets_brute_force(mp):
    """Each particle's cell is the nearest centroid of its own set, ties to the
    lowest index: brute force over the full distance matrix."""
    p = O.make_params(mp)
    x, typ = _two_set_cloud()
    rng = np.random.default_rng(5)
    kl = 30
    seeds = np.concatenate([rng.normal(size=(kl, 3)) * 6, rng.normal(size=(8, 3)) * 6])
    seeds[kl + 3] = seeds[4]                      # a protein centroid on top of a lipid one
    own = O.assign_sets(p, x, typ, seeds, kl)
    d2 = ((x[:, None, :] - seeds[None, :, :]) ** 2).sum(axis=2)
    lipid = typ == 0
    d2[np.ix_(lipid, np.arange(kl, seeds.shape[0]))] = np.inf
    d2[np.ix_(~lipid, np.arange(kl))] = np.inf
    assert np.array_equal(own, np.argmin(d2, axis=1))
    assert np.all(own[lipid] < kl) and np.all(own[~lipid] >= kl)


def test_seed_update_sets_are_set_means(mp):
    p = O.make_params(mp)
    x, typ = _two_set_cloud(seed=3)
    kl = 25
    seeds = np.concatenate([x[typ == 0][::16][:kl], x[typ != 0][::10]])
    seeds = seeds + 0.01
    own = O.assign_sets(p, x, typ, seeds, kl)
    new = O.seed_update_sets(p, x, typ, own, seeds, kl)
    for c in range(seeds.shape[0]):
        m = own == c
        if c < kl:
            m &= typ == 0
        if m.any():
            assert np.allclose(new[c], x[m].mean(axis=0), atol=1e-12), c
        else:
            assert np.array_equal(new[c], seeds[c])
    # a protein cell holding only protein members moves (the attached M-step would not move it)
    moved = [c for c in range(kl, seeds.shape[0]) if (own == c).any()]
    assert moved and all(not np.array_equal(new[c], seeds[c]) for c in moved)


def test_morton_sets_put_lipid_cells_first(mp):
    p = O.make_params(mp)
    seeds = np.array([[0.0, 0, 0], [1.0, 1, 1], [0.0, 0, 0], [1.0, 0, 0]])
    k = O.morton_sets(p, seeds, 2)
    assert k[0] == 0 and k[1] == (1 << 63) - 1
    assert k[2] == 1 << 63
    assert k[3] == (1 << 63) | sum(1 << (3 * b + 2) for b in range(21))
    x, typ = _two_set_cloud(seed=4)
    kl, kp = O.set_sizes(typ, 16)
    assert (kl, kp) == (25, 6)
    sys_ = I.System("cloud", x, np.zeros_like(x), typ, np.zeros_like(x), np.zeros_like(x),
                    np.zeros((0, 2), np.int32), np.zeros(0), np.zeros(3), np.zeros(3, np.int32), 0.22)
    seeds, owner, kl0 = O.voronoi_init_sets(p, sys_, 16, 3)
    assert kl0 == kl and seeds.shape[0] == kl + kp
    s2, o2, order = O.voronoi_update_sets(p, x, typ, seeds, kl)
    assert np.all(o2[typ == 0] < kl) and np.all(o2[typ != 0] >= kl)
    assert np.array_equal(np.sort(o2), o2[order])
    keys = O.morton_sets(p, s2, kl)
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)


def test_two_set_cell_pairs_cover_every_neighbour_pair(mp):
    """Cell pairs found from the two sets' bounding radii still contain every
    neighbour pair, lipid-protein pairs across the sets included."""
    import dataclasses
    det = I.config("tiny_detached")
    # forty protein beads pulled up to 0.9 sigma under a lipid: lipid-protein pairs
    prot = np.flatnonzero(det.type != 0)[::5][:40]
    x = det.x.copy()
    lip = np.arange(40) * 50                      # lipid ids come first
    x[prot] = det.x[lip] - 0.9 * det.n[lip]
    det = dataclasses.replace(det, x=x)
    p = O.params_for(det, mp)
    seeds, owner, kl = O.voronoi_init_sets(p, det, 16, 3)
    R = O.cell_bounds(p, det.x, owner, seeds)
    cp = O.cell_pairs(p, seeds, R, 2.6, 0.0)
    cset = set(map(tuple, cp))
    pairs = O.pairs(p, det.x, det.type)
    a, b = owner[pairs[:, 0]], owner[pairs[:, 1]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    assert all((int(u), int(v)) in cset for u, v in zip(lo, hi))
    cross = (lo < kl) & (hi >= kl)
    assert cross.sum() >= 40


# ------------------------------------------------------------------ integrator

def _energy_error(sys_, mp, dt, T):
    p = O.params_for(sys_, mp)
    n = int(round(T / dt))
    en = O.vv_run(p, sys_, dt, n)[4]
    return np.abs(en[:, 2] - en[0, 2]).max()


def test_nve_second_order(patch, mp):
    e1 = _energy_error(patch, mp, 0.01, 0.5)
    e2 = _energy_error(patch, mp, 0.005, 0.5)
    assert 3.0 < e1 / e2 < 5.5, (e1, e2)
    assert e1 < 1e-2 * patch.N


def test_time_reversal(patch, mp):
    p = O.params_for(patch, mp)
    x, v, n, w, _ = O.vv_run(p, patch, 0.01, 40)
    back = I.System("back", x, n, patch.type, -v, -w, patch.bonds, patch.r0, patch.box, patch.periodic)
    x2, v2, n2, w2, _ = O.vv_run(p, back, 0.01, 40)
    assert np.abs(x2 - patch.x).max() < 1e-9
    assert np.abs(n2 - patch.n).max() < 1e-9


def test_free_rotor(mp):
    p = O.make_params(mp)
    n0 = np.array([[1.0, 0.0, 0.0]])
    w0 = np.array([[0.0, 0.0, 0.7]])
    s = I.System("rotor", np.zeros((1, 3)), n0, np.zeros(1, np.int32), np.zeros((1, 3)), w0,
                 np.zeros((0, 2), np.int32), np.zeros(0), np.zeros(3), np.zeros(3, np.int32))
    x, v, n, w, en = O.vv_run(p, s, 0.01, 300)
    ang = 0.7 * 3.0
    assert n[0] == pytest.approx([math.cos(ang), math.sin(ang), 0.0], abs=1e-12)
    assert np.array_equal(w, w0)


def test_harmonic_dimer_period(mp):
    p = O.make_params(mp)
    r0 = 1.5
    amp = 0.05
    x = np.array([[0.0, 0, 0], [r0 + amp, 0, 0]])
    s = I.System("dimer", x, np.zeros((2, 3)), np.array([2, 2], np.int32), np.zeros((2, 3)), np.zeros((2, 3)),
                 np.array([[0, 1]], np.int32), np.array([r0]), np.zeros(3), np.zeros(3, np.int32))
    dt = 0.001
    period = 2 * math.pi / math.sqrt(2 * mp.k_bond / 1.0)
    nsteps = int(1.25 * period / dt)
    # record separations by running one step at a time (plain driver of the oracle step)
    seps = []
    cur = s
    for _ in range(nsteps):
        xx, vv, nn, ww, _ = O.vv_run(p, cur, dt, 1)
        cur = I.System("dimer", xx, nn, s.type, vv, ww, s.bonds, s.r0, s.box, s.periodic)
        seps.append(xx[1, 0] - xx[0, 0] - r0)
    seps = np.array(seps)
    # first return to the maximum: one period
    i = int(np.argmax(seps[int(0.75 * period / dt):])) + int(0.75 * period / dt)
    assert (i + 1) * dt == pytest.approx(period, rel=2e-3)
