"""Continuous-batching request loop for membrane simulations.

Requests (flat patches and vesicles of uneven sizes) arrive over time.  The loop
admits waiting requests in arrival order whenever a slot and enough device
memory are free, advances every resident system together with batched ensemble
steps, retires a request as soon as it has taken its step count, and records
per-step latency (wall time of a batched call divided by its steps, one sample
per resident request and step), arrival-to-done latency and throughput.

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


@dataclasses.dataclass
class ServeStats:
    results: List[Result]
    step_latency: np.ndarray          # seconds per step, one sample per (request, step)
    wall: float                       # first arrival -> last completion
    busy: float                       # time inside batched step calls
    particle_steps: int
    max_resident: int
    calls: int

    def summary(self) -> dict:
        lat = self.step_latency
        e2e = np.array([r.done - r.arrival for r in self.results]) if self.results else np.zeros(1)
        return {
            "requests": len(self.results),
            "particle_steps": int(self.particle_steps),
            "step_latency_ms_p50": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "step_latency_ms_p99": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "e2e_s_p50": float(np.percentile(e2e, 50)),
            "e2e_s_p99": float(np.percentile(e2e, 99)),
            "throughput_wall": self.particle_steps / self.wall if self.wall > 0 else None,
            "throughput_busy": self.particle_steps / self.busy if self.busy > 0 else None,
            "wall_s": self.wall,
            "busy_s": self.busy,
            "max_resident": self.max_resident,
            "calls": self.calls,
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
    results: List[Result] = []
    busy = 0.0
    psteps = 0
    calls = 0
    max_res = 0
    t0 = clock()
    first_arrival = pending[0]["arrival"] if pending else 0.0
    while pending or waiting or live:
        now = clock() - t0
        while pending and pending[0]["arrival"] <= now:
            waiting.append(pending.popleft())
        # requests that arrived together are staged, and their cells built in one set of
        # launches, where the executor supports it
        two_phase = hasattr(executor, "stage") and hasattr(executor, "commit")
        staged = []
        while waiting:
            req = waiting[0]
            sys_ = systems[req["id"]]
            slot = executor.stage(sys_) if two_phase else executor.admit(sys_)
            if slot is None:
                if not live and not staged:
                    raise RuntimeError(f"request {req['id']} does not fit on an empty device")
                break
            waiting.popleft()
            staged.append(slot)
            live[slot] = {"req": req, "left": int(req["steps"]), "n": int(sys_.N),
                          "admitted": None if two_phase else clock() - t0}
        if two_phase and staged:
            failed = executor.commit()
            if failed:
                raise RuntimeError(f"requests {[live[q]['req']['id'] for q in failed]} could not be admitted")
            for slot in staged:
                live[slot]["admitted"] = clock() - t0
        max_res = max(max_res, len(live))
        if not live:
            if pending:
                sleep(max(0.0, pending[0]["arrival"] - (clock() - t0)))
            continue
        nstep = min(chunk, min(r["left"] for r in live.values()))
        ts = clock()
        executor.step(nstep, dt)
        te = clock()
        calls += 1
        busy += te - ts
        per = (te - ts) / nstep
        lat_chunks.append(np.full(nstep * len(live), per))
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
    wall = (max(r.done for r in results) - first_arrival) if results else 0.0
    lat = np.concatenate(lat_chunks) if lat_chunks else np.zeros(0)
    return ServeStats(sorted(results, key=lambda r: r.req_id), lat, wall, busy, psteps, max_res, calls)
