"""The allocation-free pair export (rbc_get_pairs_noalloc) against rbc_get_pairs.

Two calls in a row on one context, the second with a smaller system, each compared
with the allocating export bit for bit (pair sets are integer data); the staging is
shared by every call on the GPU and keeps the previous call's contents, so the
second, smaller call also checks that nothing of the first leaks into it.  A set
beyond the staging's stated size is refused with RBC_ERR_CAPACITY.
"""
import dataclasses

import numpy as np
import pytest

from tests.gpu_common import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not gpu_available():
        pytest.skip("needs a GPU")
    from paper_1701_02059_amd import rbc
    rbc.lib()
    return rbc


def test_noalloc_matches_allocating_export_on_two_calls(R, mp):
    from paper_1701_02059_amd import inputs as I
    big = I.vesicle_for_lipids(40_000, seed=3)        # ~3.7e5 pairs
    small = I.config("patch")                         # 2,704 particles, periodic
    for prec in (R.RBC_MIXED, R.RBC_FP64):
        c = R.Context(mp, prec)
        for system in (big, small):
            c.set_system(system)
            c.step(5, 0.01)
            ref = c.get_pairs()
            got = c.get_pairs_noalloc()
            assert got.shape == ref.shape and got.shape[0] > 0
            assert np.array_equal(got, ref)
        c.close()


def test_noalloc_refuses_a_set_beyond_its_staging(R, mp):
    from paper_1701_02059_amd import inputs as I
    s = I.config("rbc500k")                           # ~4.4e6 pairs > 4,194,272
    c = R.Context(dataclasses.replace(mp, skin=0.5), R.RBC_MIXED)
    c.set_system(s)
    with pytest.raises(R.RbcError) as e:
        c.get_pairs_noalloc()
    assert e.value.status == R.RBC_ERR_CAPACITY
    # the allocating export still serves it, and a later small call works again
    assert c.get_pairs().shape[0] > 4_194_272
    c.set_system(I.config("patch"))
    assert np.array_equal(c.get_pairs_noalloc(), c.get_pairs())
    c.close()
