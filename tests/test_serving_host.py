"""Continuous-batching loop on the CPU with a mock executor (virtual clock)."""
import numpy as np
import pytest

from paper_1701_02059_amd import serving


class FakeSys:
    def __init__(self, n):
        self.N = n


class MockExec:
    """Slots and a byte budget like the HIP ensemble; a step costs 1 us per 1000 particles."""

    def __init__(self, clock, slots, budget):
        self.clock = clock
        self.slots = [None] * slots
        self.budget = budget
        self.used = 0
        self.steps = {}
        self.log = []

    def footprint(self, s):
        return 100 * s.N

    def admit(self, s):
        fp = self.footprint(s)
        if self.used + fp > self.budget or None not in self.slots:
            return None
        k = self.slots.index(None)
        self.slots[k] = s
        self.used += fp
        self.steps[k] = 0
        self.log.append(("admit", k, s.N))
        return k

    def step(self, n, dt):
        tot = sum(s.N for s in self.slots if s is not None)
        self.clock.t += n * (2e-5 + tot * 1e-9)
        for k, s in enumerate(self.slots):
            if s is not None:
                self.steps[k] += n

    def get_state(self, k):
        return self.steps[k]

    def retire(self, k):
        self.used -= self.footprint(self.slots[k])
        self.slots[k] = None
        self.log.append(("retire", k))


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 1e-6)


def _run(n_req, slots, budget, rate=20.0, steps=50):
    rng = np.random.default_rng(0)
    arr = np.cumsum(rng.exponential(1 / rate, n_req))
    reqs = [{"id": i, "arrival": float(arr[i]), "steps": steps} for i in range(n_req)]
    systems = {i: FakeSys(int(rng.integers(2000, 200000))) for i in range(n_req)}
    clk = Clock()
    ex = MockExec(clk, slots, budget)
    st = serving.serve(reqs, systems, ex, chunk=7, clock=clk, sleep=clk.sleep, keep_state=set(range(n_req)))
    return st, ex, systems


def test_every_request_takes_exactly_its_steps():
    st, ex, systems = _run(40, 8, 10 ** 12)
    assert len(st.results) == 40
    assert all(r.state == 50 for r in st.results)
    assert st.particle_steps == sum(s.N for s in systems.values()) * 50
    assert st.step_latency.size == 40 * 50


def test_budget_and_slots_bind():
    st, ex, systems = _run(40, 3, 100 * 250000)
    # never more than 3 resident, never over budget
    live, used, peak = set(), 0, 0
    for ev in ex.log:
        if ev[0] == "admit":
            live.add(ev[1])
            peak = max(peak, len(live))
        else:
            live.discard(ev[1])
    assert peak <= 3 and st.max_resident <= 3
    assert ex.used == 0 and all(s is None for s in ex.slots)
    # arrival order is kept for admission
    order = [r.req_id for r in sorted(st.results, key=lambda r: r.admitted)]
    assert order == sorted(order)


def test_oversized_request_raises():
    with pytest.raises(RuntimeError):
        _run(2, 2, 10)


def test_summary_fields():
    st, _, _ = _run(10, 4, 10 ** 12)
    s = st.summary()
    assert s["requests"] == 10 and s["step_latency_ms_p99"] >= s["step_latency_ms_p50"] > 0
    assert s["throughput_busy"] >= s["throughput_wall"] > 0
