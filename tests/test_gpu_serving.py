"""The serving loop on the HIP ensemble (continuous batching of the serving workload).

* Sixteen requests sampled from the serving stream (patches and vesicles of uneven
  sizes, seeded as in the benchmark; arrivals compressed so that they overlap on the
  device) go through serve() with their final states kept.  Each equals the same
  request run alone, bit for bit, and for two of them the final state's pair set
  and forces match the oracle's (pair set exactly; forces within the mixed bound).
* A slot whose state turns non-finite is frozen by the batched step: that call
  reports the error, the other slot's trajectory is unaffected (equal to its run
  alone), later calls go on without the frozen slot, and retiring it frees it.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_02059_amd import inputs as I
from paper_1701_02059_amd import serving as SV
from tests.gpu_common import PP_MIXED_TOL, check_forces, to_np

pytestmark = pytest.mark.gpu

DT = 0.01
STEPS = 40
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1701_02059_amd import rbc
    rbc.lib()
    return rbc


def _sample_requests(count=16, max_lipids=30_000):
    """The first `count` requests of the serving stream with at most max_lipids lipids,
    with STEPS steps each and arrival times compressed a hundredfold."""
    out = []
    for r in I.serving_requests(256):
        if r["nL"] <= max_lipids:
            out.append(dict(r, steps=STEPS, arrival=r["arrival"] / 100.0))
        if len(out) == count:
            break
    return out


def test_serving_results_equal_alone_runs_and_the_oracle(R, mp):
    mp = dataclasses.replace(mp, skin=0.5)
    reqs = _sample_requests()
    assert len(reqs) == 16 and len({r["kind"] for r in reqs}) == 2
    systems = {r["id"]: I.build_request(r, params=mp) for r in reqs}
    ens = R.Ensemble(mp, R.RBC_MIXED, max_slots=8)
    st = SV.serve(reqs, systems, ens, dt=DT, chunk=7, keep_state={r["id"] for r in reqs})
    ens.close()
    s = st.summary()
    assert s["requests"] == 16 and s["failed"] == 0, s
    assert s["max_resident"] > 1, s                  # they overlapped on the device
    assert st.step_latency.size == 16 * STEPS
    for res in st.results:
        assert res.error is None
        e = R.Ensemble(mp, R.RBC_MIXED, max_slots=1)
        slot = e.admit(systems[res.req_id])
        e.step(STEPS, DT)
        alone = [to_np(t) for t in e.get_state(slot)]
        e.close()
        for a, b in zip(alone, [to_np(t) for t in res.state]):
            assert np.array_equal(a, b), res.req_id
    # the two smallest requests' final states against the oracle
    for res in sorted(st.results, key=lambda r: r.n)[:2]:
        x, n, v, w = (to_np(t) for t in res.state)
        s_end = dataclasses.replace(systems[res.req_id], x=x, n=n, v=v, w=w)
        c = R.Context(mp, R.RBC_MIXED)
        c.set_system(s_end)
        F, T = (to_np(t) for t in c.forces())
        got = c.get_pairs()
        c.close()
        p = O.params_for(s_end, mp)
        assert np.array_equal(got, O.pairs(p, s_end.x, s_end.type, "grid"))
        F0, T0, _, _ = O.forces(p, s_end)
        lip = s_end.type == 0
        check_forces(F, F0, MIXED_TOL, PP_MIXED_TOL, f"request {res.req_id} F")
        check_forces(T[lip], T0[lip], MIXED_TOL, PP_MIXED_TOL, f"request {res.req_id} tau")


def test_a_failing_slot_is_frozen_and_the_rest_go_on(R, mp):
    good = I.config("patch")
    bad = dataclasses.replace(good, v=good.v.copy())
    bad.v[5, 0] = np.inf
    e = R.Ensemble(mp, R.RBC_MIXED, max_slots=4)
    a = e.admit(good)
    b = e.admit(bad)
    with pytest.raises(R.RbcError) as ei:
        e.step(2, DT)
    assert ei.value.status == R.RBC_ERR_NONFINITE
    assert e.failed() == {b: R.RBC_ERR_NONFINITE}
    with pytest.raises(R.RbcError):
        e.get_state(b)
    e.step(20, DT)                                   # the frozen slot takes no part
    got = [to_np(t) for t in e.get_state(a)]
    e.retire(b)
    assert e.failed() == {} and e.info()["live"] == 1
    e.step(5, DT)
    got5 = [to_np(t) for t in e.get_state(a)]
    e.close()
    ref = R.Ensemble(mp, R.RBC_MIXED, max_slots=1)
    s = ref.admit(good)
    ref.step(2, DT)
    ref.step(20, DT)
    ref22 = [to_np(t) for t in ref.get_state(s)]
    ref.step(5, DT)
    ref27 = [to_np(t) for t in ref.get_state(s)]
    ref.close()
    for x, y in zip(got, ref22):
        assert np.array_equal(x, y)
    for x, y in zip(got5, ref27):
        assert np.array_equal(x, y)
