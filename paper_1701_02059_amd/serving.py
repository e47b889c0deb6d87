"""Continuous-batching request loop for membrane simulations.

Requests (flat patches and vesicles of uneven sizes) arrive over time.  The loop
admits waiting requests in arrival order whenever a slot and enough device
memory are free, advances every resident system together with batched ensemble
steps, retires a request as soon as it has taken its step count, and records
per-step latency, arrival-to-done latency and throughput.

Step latency: when the executor times its steps (step_times), each resident
request gets one sample per step, the GPU interval between that step's end and the
previous one's; the first step of a call also carries the gap since the previous
call for requests resident in both, so admission work that stalls resident
requests counts.  The per-call average (call time / steps) is reported beside it.

A request that cannot be admitted (its cell build fails) or whose slot fails
during a step (the executor freezes it and lists it in failed()) is recorded with
its error, and the loop goes on with the others.  Requests must ask for at least
one step.

The executor is anything with footprint/admit/step/get_state/retire (the HIP
ensemble in paper_1701_02059_amd.rbc.Ensemble, or a mock for host-only tests).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Result:
    req_id: int
    n: int
    arrival: float
    admitted: float
    done: float
    steps: int
    state: object = None
    error: Optional[str] = None


@dataclasses.dataclass
class ServeStats:
    results: List[Result]
    step_latency: np.ndarray          # seconds per step, one sample per (request, step)
    call_latency: np.ndarray          # seconds per step as a call's average, one sample per (request, step)
    wall: float                       # first arrival -> last completion
    busy: float                       # time inside batched step calls
    particle_steps: int
    max_resident: int
    calls: int
    host_us: Optional[np.ndarray] = None   # host time per step (decisions, launches) of each call

    def summary(self) -> dict:
        lat = self.step_latency
        ok = [r for r in self.results if r.error is None]
        e2e = np.array([r.done - r.arrival for r in ok]) if ok else np.zeros(1)
        cl = self.call_latency
        return {
            "requests": len(self.results),
            "failed": len(self.results) - len(ok),
            "particle_steps": int(self.particle_steps),
            "step_latency_ms_p50": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "step_latency_ms_p99": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "call_avg_latency_ms_p50": float(np.percentile(cl, 50) * 1e3) if cl.size else None,
            "call_avg_latency_ms_p99": float(np.percentile(cl, 99) * 1e3) if cl.size else None,
            "e2e_s_p50": float(np.percentile(e2e, 50)),
            "e2e_s_p99": float(np.percentile(e2e, 99)),
            "throughput_wall": self.particle_steps / self.wall if self.wall > 0 else None,
            "throughput_busy": self.particle_steps / self.busy if self.busy > 0 else None,
            "wall_s": self.wall,
            "busy_s": self.busy,
            "max_resident": self.max_resident,
            "calls": self.calls,
            "host_us_per_step_mean": float(np.mean(self.host_us)) if self.host_us is not None and
            self.host_us.size else None,
        }


def serve(requests: List[dict], systems: Dict[int, object], executor, dt: float = 0.01, chunk: int = 10,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          keep_state: Optional[set] = None) -> ServeStats:
    """Run the request stream to completion.

    requests: dicts with id, arrival (s, relative to the start), steps.
    systems:  id -> prepared input system (built before the clock starts).
    keep_state: ids whose final state is kept (executor.get_state) in the results.
    """
    pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
    waiting: collections.deque = collections.deque()
    live: Dict[int, dict] = {}
    lat_chunks: List[np.ndarray] = []
    call_chunks: List[np.ndarray] = []
    results: List[Result] = []
    busy = 0.0
    psteps = 0
    calls = 0
    max_res = 0
    t0 = clock()
    first_arrival = pending[0]["arrival"] if pending else 0.0
    two_phase = hasattr(executor, "stage") and hasattr(executor, "commit")
    timed = hasattr(executor, "step_times")
    host_timed = hasattr(executor, "host_times")
    host_us: List[float] = []
    if timed:
        executor.step_times(True)
    prev_resident: set = set()

    def reject(req, why, admitted=None):
        now = clock() - t0
        results.append(Result(req["id"], int(systems[req["id"]].N), req["arrival"], admitted, now,
                              int(req["steps"]), None, why))

    while pending or waiting or live:
        now = clock() - t0
        while pending and pending[0]["arrival"] <= now:
            req = pending.popleft()
            if int(req["steps"]) < 1:
                reject(req, "a request must ask for at least one step")
            else:
                waiting.append(req)
        # requests that arrived together are staged, and their cells built in one set of
        # launches, where the executor supports it
        staged = []
        while waiting:
            req = waiting[0]
            sys_ = systems[req["id"]]
            try:
                slot = executor.stage(sys_) if two_phase else executor.admit(sys_)
            except Exception as e:               # the system cannot be admitted at all
                waiting.popleft()
                reject(req, f"admission failed: {e}")
                continue
            if slot is None:
                if not live and not staged:
                    raise RuntimeError(f"request {req['id']} does not fit on an empty device")
                break
            waiting.popleft()
            staged.append(slot)
            live[slot] = {"req": req, "left": int(req["steps"]), "n": int(sys_.N),
                          "admitted": None if two_phase else clock() - t0}
        if two_phase and staged:
            failed = set(executor.commit())
            for slot in staged:
                if slot in failed:
                    rec = live.pop(slot)
                    reject(rec["req"], "cell build failed")
                else:
                    live[slot]["admitted"] = clock() - t0
        max_res = max(max_res, len(live))
        if not live:
            prev_resident = set()
            if pending:
                sleep(max(0.0, pending[0]["arrival"] - (clock() - t0)))
            continue
        nstep = min(chunk, min(r["left"] for r in live.values()))
        ts = clock()
        frozen = {}
        try:
            executor.step(nstep, dt)
        except Exception:
            frozen = executor.failed() if hasattr(executor, "failed") else {}
            if not frozen:
                raise
        te = clock()
        calls += 1
        busy += te - ts
        if host_timed:
            hu = executor.host_times()[0]
            if hu >= 0:
                host_us.append(hu)
        for slot, status in frozen.items():     # slots frozen by an error in this call
            if slot in live:
                rec = live.pop(slot)
                executor.retire(slot)
                reject(rec["req"], f"failed during a step (status {status})", rec["admitted"])
        per = (te - ts) / nstep
        resident = set(live)
        if timed:
            ms, gap = executor.step_times(True)
            per_step = np.asarray(ms, dtype=np.float64)[:nstep] * 1e-3
            if per_step.size != nstep:
                per_step = np.full(nstep, per)
            for slot in resident:
                lat = per_step.copy()
                if gap > 0 and slot in prev_resident:
                    lat[0] += gap * 1e-3
                lat_chunks.append(lat)
        else:
            lat_chunks.append(np.full(nstep * len(resident), per))
        call_chunks.append(np.full(nstep * len(resident), per))
        prev_resident = resident
        for slot in list(live):
            rec = live[slot]
            rec["left"] -= nstep
            psteps += rec["n"] * nstep
            if rec["left"] == 0:
                req = rec["req"]
                state = executor.get_state(slot) if keep_state is not None and req["id"] in keep_state else None
                executor.retire(slot)
                results.append(Result(req["id"], rec["n"], req["arrival"], rec["admitted"], te - t0,
                                      int(req["steps"]), state))
                del live[slot]
                prev_resident.discard(slot)
    if timed:
        executor.step_times(False)
    wall = (max(r.done for r in results) - first_arrival) if results else 0.0
    lat = np.concatenate(lat_chunks) if lat_chunks else np.zeros(0)
    cl = np.concatenate(call_chunks) if call_chunks else np.zeros(0)
    return ServeStats(sorted(results, key=lambda r: r.req_id), lat, cl, wall, busy, psteps, max_res, calls,
                      np.asarray(host_us) if host_timed else None)
