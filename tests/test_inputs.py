"""Seeded generator: counts, geometry and velocity statistics of the synthetic workloads."""
import math

import numpy as np
import pytest

from paper_1701_02059_amd import inputs as I


def test_patch_construction():
    s = I.config("patch")
    assert s.N == 2704 and s.counts() == {"L": 2304, "S": 384, "J": 16, "bonds": 448}
    assert s.box[0] == pytest.approx(53.76) and s.box[1] == pytest.approx(46.56, abs=1e-2)
    assert list(s.periodic) == [1, 1, 0]
    lip = s.type == 0
    assert np.allclose(np.linalg.norm(s.n[lip], axis=1), 1.0)
    assert np.all(s.x[:, :2] >= 0) and np.all(s.x[:, 0] < s.box[0]) and np.all(s.x[:, 1] < s.box[1])
    assert np.abs(s.v.sum(axis=0)).max() < 1e-10
    assert np.abs(np.sum(s.w[lip] * s.n[lip], axis=1)).max() < 1e-12
    assert not s.w[~lip].any() and not s.n[~lip].any()


def test_vesicle_construction():
    s = I.config("vesicle")
    assert s.N == 124952 and s.counts() == {"L": 100000, "S": 23952, "J": 1000, "bonds": 27946}
    R = math.sqrt(100000 * 1.09 / (4 * math.pi))
    r = np.linalg.norm(s.x[:100000], axis=1)
    assert abs(r.mean() - R) < 0.01
    assert np.allclose(np.linalg.norm(s.x[100000:101000], axis=1), R - 1.2)


def test_biconcave_geometry_area_volume():
    A, V = I.evans_fung_area_volume()
    assert A == pytest.approx(134.1, abs=0.1) and V == pytest.approx(94.1, abs=0.1)


def test_rbc500k_construction():
    s = I.config("rbc500k")
    assert s.N == 499952 and s.counts()["L"] == 450000 and s.counts()["J"] == 2000
    lip = s.type == 0
    # top pole normal points up; equal-area sampling gives about one lipid per 1.09 sigma^2
    top = np.argmax(s.x[lip][:, 2] * 0 + s.n[lip][:, 2])
    assert s.n[lip][top, 2] > 0.99
    assert s.scale == pytest.approx(60.51, abs=0.01)


def test_request_stream_is_seeded():
    a = I.serving_requests(16)
    b = I.serving_requests(16)
    assert a == b
    assert all(2000 <= r["nL"] <= 200000 for r in a)
    s = I.build_request({"kind": "patch", "nL": 3000, "seed": 3})
    assert s.counts()["L"] == 54 * 54
