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


class TwoPhaseExec(MockExec):
    """Stages systems and builds them in one commit, like the HIP ensemble's two-phase
    admission; a commit costs a fixed time whatever the number of systems, and the
    systems listed in `refuse` fail their build."""

    def __init__(self, clock, slots, budget, refuse=()):
        super().__init__(clock, slots, budget)
        self.pending = []
        self.commits = []
        self.refuse = set(refuse)

    def admit(self, s):
        raise AssertionError("a two-phase executor is staged, not admitted")

    def stage(self, s):
        k = MockExec.admit(self, s)
        if k is not None:
            self.pending.append(k)
        return k

    def commit(self):
        self.clock.t += 3e-3
        self.commits.append(list(self.pending))
        failed = [k for k in self.pending if self.slots[k].N in self.refuse]
        for k in failed:
            self.retire(k)
        self.pending = []
        return failed

    def step(self, n, dt):
        assert not self.pending, "stepped with staged systems"
        super().step(n, dt)


def test_two_phase_admission_batches_arrivals():
    """Requests arriving together are staged and committed once; every request still
    takes exactly its steps, in arrival order of admission."""
    reqs = [{"id": i, "arrival": 0.0, "steps": 30} for i in range(12)]
    systems = {i: FakeSys(1000 + i) for i in range(12)}
    clk = Clock()
    ex = TwoPhaseExec(clk, 8, 10 ** 12)
    st = serving.serve(reqs, systems, ex, chunk=10, clock=clk, sleep=clk.sleep, keep_state=set(range(12)))
    assert len(st.results) == 12 and all(r.state == 30 for r in st.results)
    assert ex.commits[0] == list(range(8))              # the first eight in one commit
    assert sum(len(c) for c in ex.commits) == 12
    assert all(r.admitted is not None for r in st.results)


def test_two_phase_failed_build_is_recorded_and_the_rest_complete():
    reqs = [{"id": i, "arrival": 0.0, "steps": 10} for i in range(3)]
    systems = {i: FakeSys(1000 + i) for i in range(3)}
    clk = Clock()
    ex = TwoPhaseExec(clk, 4, 10 ** 12, refuse={1001})
    st = serving.serve(reqs, systems, ex, chunk=10, clock=clk, sleep=clk.sleep, keep_state={0, 2})
    by = {r.req_id: r for r in st.results}
    assert by[1].error == "cell build failed" and by[1].state is None
    assert by[0].error is None and by[0].state == 10
    assert by[2].error is None and by[2].state == 10
    assert st.summary()["failed"] == 1
    assert ex.used == 0 and all(s is None for s in ex.slots)


class FreezingExec(MockExec):
    """Freezes the slot of the system of size `bad` at its first step call, the way the
    HIP ensemble freezes a slot whose lists overflow: the call raises, the other slots
    have advanced, and failed() lists the frozen slot until it is retired."""

    def __init__(self, clock, slots, budget, bad):
        super().__init__(clock, slots, budget)
        self.bad = bad
        self.frozen = {}

    def step(self, n, dt):
        tot = sum(s.N for s in self.slots if s is not None)
        self.clock.t += n * (2e-5 + tot * 1e-9)
        for k, s in enumerate(self.slots):
            if s is None or k in self.frozen:
                continue
            if s.N == self.bad:
                self.frozen[k] = 5
            else:
                self.steps[k] += n
        if self.frozen:
            raise RuntimeError("capacity exceeded (slot frozen)")

    def failed(self):
        return dict(self.frozen)

    def retire(self, k):
        self.frozen.pop(k, None)
        super().retire(k)


def test_a_slot_failing_during_a_step_is_retired_and_the_rest_complete():
    reqs = [{"id": i, "arrival": 0.001 * i, "steps": 40} for i in range(6)]
    systems = {i: FakeSys(3000 + i) for i in range(6)}
    clk = Clock()
    ex = FreezingExec(clk, 4, 10 ** 12, bad=3002)
    st = serving.serve(reqs, systems, ex, chunk=10, clock=clk, sleep=clk.sleep, keep_state=set(range(6)))
    by = {r.req_id: r for r in st.results}
    assert len(by) == 6
    assert by[2].error is not None and "failed during a step" in by[2].error
    assert all(by[i].error is None and by[i].state == 40 for i in (0, 1, 3, 4, 5))
    assert ex.used == 0 and all(s is None for s in ex.slots)


def test_a_step_error_without_a_frozen_slot_still_raises():
    class Broken(MockExec):
        def step(self, n, dt):
            raise RuntimeError("device lost")

        def failed(self):
            return {}

    reqs = [{"id": 0, "arrival": 0.0, "steps": 10}]
    clk = Clock()
    with pytest.raises(RuntimeError):
        serving.serve(reqs, {0: FakeSys(1000)}, Broken(clk, 2, 10 ** 12), clock=clk, sleep=clk.sleep)


def test_requests_without_steps_are_refused():
    reqs = [{"id": 0, "arrival": 0.0, "steps": 0}, {"id": 1, "arrival": 0.0, "steps": -3},
            {"id": 2, "arrival": 0.0, "steps": 5}]
    systems = {i: FakeSys(1000) for i in range(3)}
    clk = Clock()
    ex = MockExec(clk, 4, 10 ** 12)
    st = serving.serve(reqs, systems, ex, chunk=10, clock=clk, sleep=clk.sleep, keep_state={2})
    by = {r.req_id: r for r in st.results}
    assert by[0].error and by[1].error and by[2].error is None and by[2].state == 5
    assert [ev[0] for ev in ex.log] == ["admit", "retire"]          # only the valid request was admitted


class TimedExec(MockExec):
    """Reports per-step times like the HIP ensemble's step_times: step q of a call
    takes q + 1 ms, and every call after the first follows a 10 ms gap."""

    def __init__(self, clock, slots, budget):
        super().__init__(clock, slots, budget)
        self.last = (np.zeros(0), -1.0)
        self.ncalls = 0

    def step(self, n, dt):
        super().step(n, dt)
        self.last = (np.arange(1, n + 1, dtype=np.float64), 10.0 if self.ncalls else -1.0)
        self.ncalls += 1

    def step_times(self, enable=True):
        return self.last


def test_step_latency_comes_from_per_step_times_and_carries_gaps():
    reqs = [{"id": 0, "arrival": 0.0, "steps": 6}]
    clk = Clock()
    ex = TimedExec(clk, 2, 10 ** 12)
    st = serving.serve(reqs, {0: FakeSys(1000)}, ex, chunk=3, clock=clk, sleep=clk.sleep)
    # two calls of 3 steps: 1, 2, 3 ms, then 1 + 10 (the gap), 2, 3 ms
    assert np.allclose(np.sort(st.step_latency * 1e3), np.sort([1, 2, 3, 11, 2, 3]))
    assert st.call_latency.size == 6
