"""Pins of the oracle's pair laws against mathematics, not against itself.

Lipid-lipid law: finite differences of U (force and torque), closed values at
r_min, zero beyond r_c, continuity, symmetry and invariance properties, and the
per-pair momentum / angular-momentum identities.  WCA and bonds: textbook
closed forms and finite differences.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_02059_amd.inputs import ModelParams


def _rand_unit(rng, k=1):
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rot(axis, ang):
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def _params(st0=0.0):
    mp = ModelParams(sin_theta0=st0)
    return O.make_params(mp), mp


@pytest.mark.parametrize("st0", [0.0, 0.1])
def test_lipid_force_is_minus_gradient(st0):
    p, mp = _params(st0)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(200):
        r = rng.uniform(0.85, mp.r_c - 1e-3)
        d = _rand_unit(rng)[0] * r
        ni, nj = _rand_unit(rng, 2)
        U, Fi, ti, tj = O.pair_lipid(p, d, ni, nj)
        g = np.zeros(3)
        for a in range(3):
            dp, dm = d.copy(), d.copy()
            dp[a] += h
            dm[a] -= h
            g[a] = (O.pair_lipid(p, dp, ni, nj)[0] - O.pair_lipid(p, dm, ni, nj)[0]) / (2 * h)
        scale = max(1.0, np.linalg.norm(Fi))
        assert np.allclose(Fi, -g, rtol=0, atol=1e-7 * scale), (r, Fi, -g)


@pytest.mark.parametrize("st0", [0.0, 0.1])
def test_lipid_torque_is_minus_rotation_derivative(st0):
    p, mp = _params(st0)
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(200):
        r = rng.uniform(0.85, mp.r_c - 1e-3)
        d = _rand_unit(rng)[0] * r
        ni, nj = _rand_unit(rng, 2)
        U, Fi, ti, tj = O.pair_lipid(p, d, ni, nj)
        for which, tq in ((0, ti), (1, tj)):
            g = np.zeros(3)
            for a in range(3):
                ax = np.eye(3)[a]
                Rp, Rm = _rot(ax, h), _rot(ax, -h)
                if which == 0:
                    up = O.pair_lipid(p, d, Rp @ ni, nj)[0]
                    um = O.pair_lipid(p, d, Rm @ ni, nj)[0]
                else:
                    up = O.pair_lipid(p, d, ni, Rp @ nj)[0]
                    um = O.pair_lipid(p, d, ni, Rm @ nj)[0]
                g[a] = (up - um) / (2 * h)
            scale = max(1.0, np.linalg.norm(tq))
            assert np.allclose(tq, -g, rtol=0, atol=1e-7 * scale)


def test_lipid_closed_values_at_rmin():
    p, mp = _params(0.0)
    r = mp.r_min
    ex, ez = np.array([1.0, 0, 0]), np.array([0, 0, 1.0])
    d = ex * r
    # normals parallel, perpendicular to the separation: the sheet minimum, -eps
    assert O.pair_lipid(p, d, ez, ez)[0] == pytest.approx(-mp.eps, abs=1e-14)
    # antiparallel: (2 mu - 1) eps
    assert O.pair_lipid(p, d, ez, -ez)[0] == pytest.approx((2 * mp.mu - 1) * mp.eps, abs=1e-13)
    # stacked along the separation: (mu - 1) eps
    assert O.pair_lipid(p, d, ex, ex)[0] == pytest.approx((mp.mu - 1) * mp.eps, abs=1e-13)
    # with a spontaneous-curvature angle: n_i = z, n_j = r-hat -> a = s0 - s0^2
    p1, mp1 = _params(0.1)
    a = 0.1 - 0.01
    assert O.pair_lipid(p1, d, ez, ex)[0] == pytest.approx(-(1 + mp1.mu * (a - 1)) * mp1.eps, abs=1e-13)
    # and the mirror choice n_i = r-hat, n_j = z -> a = -s0 - s0^2
    a2 = -0.1 - 0.01
    assert O.pair_lipid(p1, d, ex, ez)[0] == pytest.approx(-(1 + mp1.mu * (a2 - 1)) * mp1.eps, abs=1e-13)


def test_lipid_closed_values_repulsive_and_attractive_branches():
    p, mp = _params(0.0)
    ez = np.array([0, 0, 1.0])
    # aligned sheet (a = 1, phi = 1): U = u_R(r) below r_min, u_A(r) above
    for r in (0.9, 1.0, 1.05):
        q = (mp.r_min / r) ** 2
        assert O.pair_lipid(p, np.array([r, 0, 0]), ez, ez)[0] == pytest.approx(q * q - 2 * q, abs=1e-13)
    for r in (1.3, 1.9, 2.5):
        x = 0.5 * math.pi * (r - mp.r_min) / (mp.r_c - mp.r_min)
        assert O.pair_lipid(p, np.array([0, r, 0]), ez, ez)[0] == pytest.approx(-math.cos(x) ** 8, abs=1e-14)
    # antiparallel (a = -1, phi = 1 - 2 mu): U = u_R + 2 mu eps below r_min
    r = 1.0
    q = (mp.r_min / r) ** 2
    assert O.pair_lipid(p, np.array([r, 0, 0]), ez, -ez)[0] == pytest.approx(q * q - 2 * q + 2 * mp.mu, abs=1e-12)


def test_lipid_zero_beyond_cutoff_and_continuity():
    p, mp = _params(0.0)
    rng = np.random.default_rng(3)
    for _ in range(50):
        ni, nj = _rand_unit(rng, 2)
        e = _rand_unit(rng)[0]
        for r in (mp.r_c + 1e-12, mp.r_c + 0.1, 5.0):
            U, Fi, ti, tj = O.pair_lipid(p, e * r, ni, nj)
            assert U == 0.0 and not Fi.any() and not ti.any() and not tj.any()
        # at r_c itself (up to rounding of |e r|) U and F vanish to all practical precision
        U, Fi, ti, tj = O.pair_lipid(p, e * mp.r_c, ni, nj)
        assert abs(U) < 1e-100 and np.abs(Fi).max() < 1e-80
        # continuity of U and F at r_c and r_min
        for r0 in (mp.r_c, mp.r_min):
            ua, fa = O.pair_lipid(p, e * (r0 - 1e-9), ni, nj)[:2]
            ub, fb = O.pair_lipid(p, e * (r0 + 1e-9), ni, nj)[:2]
            assert abs(ua - ub) < 1e-7
            assert np.allclose(fa, fb, atol=1e-6)


@pytest.mark.parametrize("st0", [0.0, 0.1])
def test_lipid_symmetries_and_identities(st0):
    p, mp = _params(st0)
    rng = np.random.default_rng(4)
    for _ in range(200):
        r = rng.uniform(0.85, mp.r_c - 1e-3)
        d = _rand_unit(rng)[0] * r
        ni, nj = _rand_unit(rng, 2)
        U, Fi, ti, tj = O.pair_lipid(p, d, ni, nj)
        # exchange i <-> j: same energy, opposite force, torques swap
        U2, Fj, tj2, ti2 = O.pair_lipid(p, -d, nj, ni)
        assert U2 == pytest.approx(U, abs=1e-12)
        assert np.allclose(Fj, -Fi, atol=1e-12)
        assert np.allclose(ti2, ti, atol=1e-12) and np.allclose(tj2, tj, atol=1e-12)
        # angular momentum: r_ij x F_i + tau_i + tau_j = 0
        assert np.allclose(np.cross(d, Fi) + ti + tj, 0.0, atol=1e-12)
        # torques are perpendicular to their orientations
        assert abs(ti @ ni) < 1e-12 and abs(tj @ nj) < 1e-12
        # global rotation
        Q = _rot(_rand_unit(rng)[0], rng.uniform(0, 2 * math.pi))
        U3, F3, t3, t4 = O.pair_lipid(p, Q @ d, Q @ ni, Q @ nj)
        assert U3 == pytest.approx(U, abs=1e-12)
        assert np.allclose(F3, Q @ Fi, atol=1e-11) and np.allclose(t3, Q @ ti, atol=1e-11)
        if st0 == 0.0:
            # head-tail symmetry without spontaneous curvature
            assert O.pair_lipid(p, d, -ni, -nj)[0] == pytest.approx(U, abs=1e-12)


def test_wca_closed_form_and_gradient():
    p, mp = _params()
    rcut = 2 ** (1 / 6)
    U, F = O.pair_wca(p, np.array([rcut, 0, 0]))
    assert U == 0.0 and not F.any()
    U, F = O.pair_wca(p, np.array([1.0, 0, 0]))
    assert U == pytest.approx(1.0, abs=1e-14) and F == pytest.approx([24.0, 0, 0], abs=1e-12)
    U, F = O.pair_wca(p, np.array([rcut - 1e-9, 0, 0]))
    assert abs(U) < 1e-12 and np.linalg.norm(F) < 1e-6
    rng = np.random.default_rng(5)
    h = 1e-7
    for _ in range(100):
        d = _rand_unit(rng)[0] * rng.uniform(0.9, rcut - 1e-3)
        U, F = O.pair_wca(p, d)
        g = np.array([(O.pair_wca(p, d + h * e)[0] - O.pair_wca(p, d - h * e)[0]) / (2 * h) for e in np.eye(3)])
        assert np.allclose(F, -g, rtol=1e-6, atol=1e-6)


def test_bond_closed_form_and_gradient():
    p, mp = _params()
    U, F = O.bond(p, np.array([0, 0, 1.5]), 1.0)
    assert U == pytest.approx(0.5 * mp.k_bond * 0.25) and F == pytest.approx([0, 0, -mp.k_bond * 0.5])
    U, F = O.bond(p, np.array([0.3, 0, 0]), 1.0)
    assert F[0] == pytest.approx(mp.k_bond * 0.7)
    rng = np.random.default_rng(6)
    h = 1e-7
    for _ in range(50):
        d = _rand_unit(rng)[0] * rng.uniform(0.5, 2.5)
        r0 = rng.uniform(0.8, 1.5)
        U, F = O.bond(p, d, r0)
        g = np.array([(O.bond(p, d + h * e, r0)[0] - O.bond(p, d - h * e, r0)[0]) / (2 * h) for e in np.eye(3)])
        assert np.allclose(F, -g, atol=1e-7)


def test_min_image_and_exact_distance():
    mp = ModelParams()
    p = O.make_params(mp, box=(10.0, 8.0, 0.0), periodic=(1, 1, 0))
    d2, d = O.dist2(p, np.array([9.5, 0.5, 0.0]), np.array([0.5, 7.5, 3.0]))
    assert d == pytest.approx([-1.0, 1.0, -3.0])
    assert d2 == 11.0
    # half-box tie rounds half to even: d/L = 0.5 -> k = 0, 1.5 -> k = 2
    _, d = O.dist2(p, np.array([5.0, 0, 0]), np.array([0.0, 0, 0]))
    assert d[0] == 5.0
    _, d = O.dist2(p, np.array([15.0, 0, 0]), np.array([0.0, 0, 0]))
    assert d[0] == -5.0
    # the squared distance is the left-to-right sum of separately rounded squares
    a = np.array([0.1, 0.7, 1.3])
    b = np.array([1.9, 0.2, -0.4])
    p0 = O.make_params(mp)
    d2, d = O.dist2(p0, a, b)
    dd = a - b
    assert d2 == (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
