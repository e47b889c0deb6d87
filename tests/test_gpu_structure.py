"""Velocity quenching of generated structures (Initial structure generation
section), GPU path vs the FP64 oracle through the C ABI.

A structure sampled on a mesh overlaps; quenching relaxes it.  The quench is
checked as an FP64 trajectory against the oracle's, for bitwise call-chunking
neutrality, and on a generated Evans-Fung cell: the energy falls, the overlaps
go, and the relaxed cell then runs NVE dynamics with its energy conserved.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_02059_amd import inputs as I
from paper_1701_02059_amd import structure as G
from tests.gpu_common import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1701_02059_amd import rbc
    rbc.lib()
    return rbc


@pytest.fixture(scope="module")
def sphere_gen():
    v, t = I.sphere_mesh(400, 40.0)
    s, ident, face = G.generate(v, t, G.GenParams(seed=2))
    return s


def _qp(mp):
    return dataclasses.replace(mp, quench=1, quench_max=0.05)


def test_quench_trajectory_fp64(R, mp, sphere_gen):
    """FP64 quenching against the oracle.  The projection v <- (v.F / |F|^2) F has
    condition number |v| / |F|: on a bead whose large pair forces nearly cancel,
    the last-bit differences of the two sides' force sums grow by that factor
    each step (measured: 7e-15 in x after one step, 4e-11 after 10, 6e-9 after
    30, in a few spectrin beads).  So positions are held to 1e-9 over 10 steps,
    and over 30 steps the energy to 1e-9 and positions to 1e-7."""
    m = _qp(mp)
    p, e = O.params_for(sphere_gen, m), O.make_ext(m)
    for nst, xtol in ((10, 1e-9), (30, 1e-7)):
        x0, v0, n0, w0, en = O.vv_run_ext(p, e, sphere_gen, 0.01, nst)
        c = R.Context(m, R.RBC_FP64)
        c.set_system(sphere_gen)
        c.step(nst, 0.01)
        x, n, v, w = (to_np(t) for t in c.get_state())
        E = c.energy()
        c.close()
        assert np.abs(x - x0).max() < xtol, nst
        assert np.abs(n - n0).max() < xtol, nst
        assert E[0] == pytest.approx(en[-1, 1], rel=1e-9), nst
    assert en[-1, 1] < 0.2 * en[0, 1]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_quench_chunking_is_bitwise_neutral(R, mp, sphere_gen, prec):
    m = _qp(mp)
    pr = R.RBC_FP64 if prec == "fp64" else R.RBC_MIXED
    outs = []
    for split in ((40,), (10, 10, 10, 10), (39, 1)):
        c = R.Context(m, pr)
        c.set_system(sphere_gen)
        for k in split:
            c.step(k, 0.01)
        outs.append([to_np(t) for t in c.get_state()])
        c.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def test_generated_cell_quench_then_dynamics(R, mp):
    """A 100k-particle cell generated on an Evans-Fung mesh: 600 mixed quenching steps
    take the energy from positive (overlaps) to a bound sheet and every particle
    more than 0.8 sigma from the next; the relaxed cell, given thermal velocities,
    then runs 500 NVE steps conserving energy."""
    from scipy.spatial import cKDTree
    v, t = I.evans_fung_mesh(500, 90_000 * I.LIPID_AREA)
    s, ident, face = G.generate(v, t, G.GenParams(seed=4))
    c = R.Context(_qp(mp), R.RBC_MIXED)
    c.set_system(s)
    U0 = c.energy()[0]
    c.step(600, 0.01)
    U1 = c.energy()[0]
    x, n, _, _ = (to_np(a) for a in c.get_state())
    c.close()
    assert U0 > 0 and U1 < 0, (U0, U1)
    assert cKDTree(x).query(x, k=2)[0][:, 1].min() > 0.8
    # thermal velocities, then dynamics
    rng = np.random.default_rng(0)
    relaxed = dataclasses.replace(s, x=x, n=n, v=rng.normal(0, np.sqrt(0.22), x.shape), w=np.zeros_like(x))
    lip = s.type == 0
    w = rng.normal(0, np.sqrt(0.22), x.shape)
    w[lip] -= np.einsum("ij,ij->i", w[lip], n[lip])[:, None] * n[lip]
    w[~lip] = 0
    relaxed = dataclasses.replace(relaxed, w=w)
    c = R.Context(mp, R.RBC_MIXED)
    c.set_system(relaxed)
    E0 = c.energy()[3]
    c.step(500, 0.01)
    E1 = c.energy()[3]
    c.close()
    assert abs(E1 - E0) / s.N < 5e-3, (E0, E1)
