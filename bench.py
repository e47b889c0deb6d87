#!/usr/bin/env python
"""Benchmark: particle-steps/s of the whole-cell workload on one MI355X.

Workload: the whole red cell, 3,999,952 particles (3.6M lipids on an Evans-Fung
biconcave surface, 16,000 junctions and 383,952 spectrin beads in a triangular
network of 8-bead chains under it), NVE velocity Verlet with dt = 0.01 tau and
Voronoi cell updates every 100 steps (earlier when the skin demands).  The
headline value is mixed precision (FP32 pair arithmetic, FP64 positions,
integration and sums); plain FP64 is reported beside it, with the pair-force
kernel's roofline fraction, the FP64 CPU oracle timed on this host's cores, and
the continuous-batching serving ensemble (p50/p99 step latency).

One JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DT = 0.01
# Algorithmic work of the timed force kernel, which also applies the closing
# half-kick, the next opening half-kick and the drift.  Flops: operation counts
# of the pair laws as written, once per unordered pair (add/sub/mul 1, FMA 2,
# sqrt/rsqrt/sin/cos/div 1), without the energy and virial terms, which the timed
# kernel does not compute.
FLOPS_LIPID_PAIR = 139      # per unordered lipid pair: F_i, F_j, tau_i, tau_j and the distance test
FLOPS_WCA_PAIR = 29         # per unordered pair with a protein bead
FLOPS_BOND = 19             # per bond
# Bytes: the state read and written once per step.  Lipid: read x (24) + type (1) + FP32 n
# for the partner stage (12) + v, omega, n (72); write x, v, n, omega (96) + FP32 n (12).
# Protein bead: read x (24) + type (1) + v (24); write x, v (48).
BYTES_LIPID_STEP = 217
BYTES_PROTEIN_STEP = 97
PEAK_FP32 = 157.3           # TFLOP/s, MI355X FP32 vector (published; counts packed FP32)
PEAK_FP64 = 78.6            # TFLOP/s, MI355X FP64 vector
PEAK_HBM = 8000.0           # GB/s
# HBM traffic of that kernel per launch at the whole-cell workload, mixed precision,
# skins 0.65 and 0.15: rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB -> bytes; factors from a
# plain 512 MiB device copy), valid only for the kernel sources whose digest is given.
FORCE_TRAFFIC = {"sources_sha256": "f735d1ee4833da80", "skin": 0.65, "inner_skin": 0.15,
                 "bytes": 1512659236, "fetch_kib": 504500, "write_kib": 468206,
                 "valu_insts": 181583857}   # SQ_INSTS_VALU per launch (wavefront instructions)
BYTES_BUILD_READ = 25       # list build: position (3 x 8 B) and type (1 B) of every particle, read once
CU_COUNT, SIMDS_PER_CU, CLOCK_GHZ = 256, 4, 2.4
KERNEL_SOURCES = ("paper_1701_02059_amd/csrc/k_force.hip", "paper_1701_02059_amd/csrc/k_cells.hip",
                  "paper_1701_02059_amd/csrc/rbc_dev.h")


def workload_shape(name: str) -> str:
    """What the named synthetic workload is, for the JSON line's config."""
    base = name[: -len("_detached")] if name.endswith("_detached") else name
    shape = {"patch": "flat periodic membrane patch", "vesicle": "spherical vesicle",
             "tiny": "small spherical vesicle"}.get(base, "whole-RBC biconcave cell")
    return shape + (", detached cytoskeleton" if base != name else "")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pair_counts(ctx, system):
    pairs = ctx.get_pairs()
    t = system.type
    ll = int(np.sum((t[pairs[:, 0]] == 0) & (t[pairs[:, 1]] == 0)))
    return ll, int(pairs.shape[0] - ll)


def timed_run(R, mp, system, precision, steps, warmup, label):
    import torch
    ctx = R.Context(mp, precision)
    t0 = time.perf_counter()
    ctx.set_system(system)
    log(f"[{label}] cells built in {time.perf_counter() - t0:.2f} s: {ctx.stats()}")
    ctx.step(warmup, DT)
    torch.cuda.synchronize()
    ctx.force_timing(True)
    st0 = ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps, DT)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    host_us, wait_us = ctx.host_times()
    build_ms, builds = ctx.build_timing()
    avg_ms, launches = ctx.force_timing(False)
    st1 = ctx.stats()
    e = ctx.energy()
    ms = (t1 - t0) * 1e3 / steps
    out = {"seconds": t1 - t0, "steps": steps, "ms_per_step": ms,
           "particle_steps_per_s": system.N * steps / (t1 - t0),
           "force_ms": avg_ms, "force_launches": launches,
           # everything else a step pays for, amortised: cell updates, list builds,
           # prunes, the drift statistics and the host loop
           "other_ms_per_step": ms - avg_ms,
           "cell_updates": st1["cell_updates"] - st0["cell_updates"],
           "list_rebuilds": st1["rebuilds"] - st0["rebuilds"],
           "early_rebuilds": st1["early_rebuilds"] - st0["early_rebuilds"],
           "prunes": st1["prunes"] - st0["prunes"],
           "max_list_rows": st1["max_list_rows"],
           # the list-build kernel (lists and pruned lists of a build), HIP events
           "build_kernel_ms": build_ms, "build_launches": builds,
           # host time per step in the step loop: deciding and launching, and waiting for
           # the drift statistics of the step before
           "host_us_per_step": host_us, "host_wait_us_per_step": wait_us,
           "energy": e.tolist()}
    log(f"[{label}] {steps} steps in {t1 - t0:.3f} s -> {out['particle_steps_per_s']:.4g} particle-steps/s, "
        f"force kernel {avg_ms * 1e3:.1f} us avg over {launches} launches, {out['cell_updates']} cell updates, "
        f"{out['list_rebuilds']} list builds, {out['prunes']} prunes")
    return ctx, out


def list_output_bytes(ctx):
    """What a list build of the current state writes, in bytes: the 16-bit lists and
    pruned lists as stored (ELL rows of each 64-particle chunk, padding included) and
    the 32-bit stage and pruned-stage slots of each 256-particle block."""
    nlk = ctx.debug_array(8).view(np.int32).astype(np.int64)
    scount = ctx.debug_array(9).view(np.int32).astype(np.int64)
    iscount = ctx.debug_array(12).view(np.int32).astype(np.int64)
    ilk = ctx.debug_array(13).view(np.int32).astype(np.int64)
    return int(2 * 64 * (nlk.sum() + ilk.sum()) + 4 * (np.maximum(scount, 0).sum() + np.maximum(iscount, 0).sum()))


def build_roofline(mixed, list_bytes, n):
    """The list-build kernel against the HBM roofline: its algorithmic bytes are every
    particle's position and type read once (BYTES_BUILD_READ per particle) plus what it
    writes (list_output_bytes)."""
    if not mixed["build_launches"]:
        return None
    b = BYTES_BUILD_READ * n + list_bytes
    t = mixed["build_kernel_ms"] * 1e-3
    return {"kernel": "k_nlist (candidate union, stage, lists and pruned lists of a build)", "bound": "hbm",
            "avg_launch_ms": round(mixed["build_kernel_ms"], 4), "launches_timed": mixed["build_launches"],
            "algorithmic_bytes_per_launch": b, "achieved": round(b / t / 1e9, 3), "peak": PEAK_HBM,
            "unit": "GB/s", "frac": round(b / t / 1e9 / PEAK_HBM, 4),
            "roofline_time_us": round(b / (PEAK_HBM * 1e9) * 1e6, 2)}


def _oracle_steps(system, mp, threads):
    """Seconds per velocity-Verlet step of the FP64 oracle: a 3-step run minus a 1-step
    run, so the initial force evaluation is not counted."""
    from oracle import oracle as O
    p = O.params_for(system, mp)
    t0 = time.perf_counter()
    O.vv_run(p, system, DT, 1, nthreads=threads)
    t1 = time.perf_counter()
    O.vv_run(p, system, DT, 3, nthreads=threads)
    t2 = time.perf_counter()
    per_step = ((t2 - t1) - (t1 - t0)) / 2.0
    if per_step <= 0:
        per_step = (t2 - t1) / 4.0
    return per_step, t2 - t0


def host_cpu():
    """Model name and usable core count of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(system, mp):
    """The FP64 oracle on this host: on all usable cores on the full cell, and on one core
    on an eighth of the same cell (the particles of smallest x, an open cap of the
    membrane with the same local density), in particle-steps/s."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    per_step, spent = _oracle_steps(system, mp, threads)
    cut = np.sort(system.x[:, 0])[system.N // 8]
    piece = system.subset(np.flatnonzero(system.x[:, 0] < cut))
    per1, spent1 = _oracle_steps(piece, mp, 1)
    return {"value": system.N / per_step, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"2 velocity-Verlet steps of the full {system.N:,}-particle cell (3-step minus 1-step run, "
                      f"{spent:.1f} s of CPU work)", "seconds_per_step": per_step, "host": host_cpu(),
            "one_core": {"value": piece.N / per1, "unit": "particle-steps/s", "cores": 1,
                         "sample": f"2 steps of the {piece.N:,} particles of smallest x of the same cell (an "
                                   f"eighth; 3-step minus 1-step run, {spent1:.1f} s)"}}


def config_leg(R, mp, system, steps, frames, oracle_steps, label):
    """A plain-FP64 workload: GPU throughput over `steps` timed steps, the NVE energy
    drift over the same number of steps sampled at `frames` frames, and the FP64
    oracle's rate on this host over `oracle_steps` steps."""
    from oracle import oracle as O
    ctx, r = timed_run(R, mp, system, R.RBC_FP64, steps, 0, label)
    ctx.close()
    r.pop("energy", None)
    ctx = R.Context(mp, R.RBC_FP64)
    ctx.set_system(system)
    e = [ctx.energy()[3]]
    for _ in range(frames):
        ctx.step(steps // frames, DT)
        e.append(ctx.energy()[3])
    ctx.close()
    e = np.array(e)
    r["nve"] = {"E0": float(e[0]), "max_abs_dE": float(np.max(np.abs(e - e[0]))),
                "max_abs_dE_per_particle": float(np.max(np.abs(e - e[0])) / system.N),
                "drift_per_particle_per_1e4_steps": float((e[-1] - e[0]) / system.N * 1e4 / steps),
                "frames": frames + 1}
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    p = O.params_for(system, mp)
    t0 = time.perf_counter()
    O.vv_run(p, system, DT, oracle_steps, nthreads=threads)
    t1 = time.perf_counter()
    r["oracle"] = {"value": system.N * oracle_steps / (t1 - t0), "unit": "particle-steps/s", "cores": threads,
                   "sample": f"{oracle_steps} velocity-Verlet steps (with the initial force evaluation), "
                             f"{t1 - t0:.1f} s"}
    r["particles"] = system.N
    log(f"[{label}] nve {r['nve']} oracle {r['oracle']}")
    return r


def detached_run(R, mp, workload, steps, warmup):
    """The same cell with its cytoskeleton detached (3 sigma under the sheet, every
    second junction tethered): mixed-precision throughput with a separate protein
    cell set and with the proteins sharing the lipids' cells."""
    from paper_1701_02059_amd import inputs as I
    name = f"{workload}_detached"
    system = I.config(name)
    out = {"workload": name, "particles": system.N}
    for key, pc in (("separate_cells", 1), ("shared_cells", 0)):
        m = dataclasses.replace(mp, protein_cells=pc)
        try:
            ctx, r = timed_run(R, m, system, R.RBC_MIXED, steps, warmup, f"detached {key}")
            st = ctx.stats()
            ctx.close()
            r.update(cells=st["cells"], lipid_cells=st["lipid_cells"], max_cell_pairs=st["max_cell_pairs"])
            r.pop("energy", None)
        except R.RbcError as e:
            r = {"error": str(e)}
        out[key] = r
    return out


def ext_run(R, mp, system, steps, warmup):
    """The same cell with the harmonic volume constraint (V0 = the loaded volume) and
    the Langevin thermostat on translations and lipid rotations."""
    m = dataclasses.replace(mp, vol_k=10.0, vol_target=0.0, kT=0.22, gamma=1.0, gamma_rot=1.0, seed=1)
    ctx, r = timed_run(R, m, system, R.RBC_MIXED, steps, warmup, "volume+thermostat")
    ctx.close()
    r.pop("energy", None)
    r["settings"] = {"vol_k": m.vol_k, "gamma": m.gamma, "gamma_rot": m.gamma_rot, "kT": m.kT}
    return r


def structure_run(R, mp, warmup, steps=1000):
    """A cell generated on a 2,000-vertex Evans-Fung mesh (about 500k particles),
    relaxed by velocity quenching: quench throughput and the energy it removes."""
    from paper_1701_02059_amd import inputs as I
    from paper_1701_02059_amd import structure as G
    t0 = time.perf_counter()
    v, t = I.evans_fung_mesh(2000, 450_000 * I.LIPID_AREA)
    system, ident, _ = G.generate(v, t, G.GenParams(seed=0))
    gen_s = time.perf_counter() - t0
    log(f"[structure] generated {system.N:,} particles on {t.shape[0]:,} triangles in {gen_s:.1f} s")
    m = dataclasses.replace(mp, quench=1, quench_max=0.05)
    ctx = R.Context(m, R.RBC_MIXED)
    ctx.set_system(system)
    U0 = float(ctx.energy()[0])
    ctx.close()
    ctx, r = timed_run(R, m, system, R.RBC_MIXED, steps, warmup, "quench")
    U1 = float(ctx.energy()[0])
    ctx.close()
    r.pop("energy", None)
    r.update(particles=system.N, generation_s=gen_s, U_start=U0, U_end=U1,
             quench_steps=steps + warmup)
    return r


def serving_run(R, mp, count, rate, steps, saturated=False, graphs=False):
    from paper_1701_02059_amd import inputs as I
    from paper_1701_02059_amd import serving as SV
    reqs = I.serving_requests(count, rate=rate, steps=steps)
    if saturated:
        for r in reqs:
            r["arrival"] = 0.0
    t0 = time.perf_counter()
    systems = {r["id"]: I.build_request(r, params=mp) for r in reqs}
    log(f"[serving] built {count} requests in {time.perf_counter() - t0:.1f} s "
        f"({sum(s.N for s in systems.values()):,} particles)")
    ens = R.Ensemble(mp, R.RBC_MIXED, max_slots=128, hbm_budget=96 << 30)
    ens.set_graphs(graphs)
    st = SV.serve(reqs, systems, ens, dt=DT, chunk=10)
    ens.close()
    s = st.summary()
    log(f"[serving{' saturated' if saturated else ''}{' graphs' if graphs else ''}] {s}")
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--workload", default="rbc4m")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-detached", action="store_true")
    ap.add_argument("--no-ext", action="store_true")
    ap.add_argument("--no-structure", action="store_true")
    ap.add_argument("--detached-steps", type=int, default=500)
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-steps", type=int, default=500)
    ap.add_argument("--skin", type=float, default=0.65,
                    help="Verlet skin of the full lists (sigma); measured optimum for the whole cell")
    ap.add_argument("--inner-skin", type=float, default=0.15,
                    help="buffer of the pruned lists the step kernel walks (sigma)")
    ap.add_argument("--no-configs", action="store_true", help="skip the FP64 patch and vesicle legs")
    ap.add_argument("--cell-target", type=int, default=16, help="mean lipids per Voronoi cell")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1701_02059_amd import inputs as I
    from paper_1701_02059_amd import rbc as R
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    R.lib()
    mp = I.ModelParams(skin=args.skin, inner_skin=args.inner_skin, cell_target=args.cell_target)
    t0 = time.perf_counter()
    system = I.config(args.workload)
    log(f"[gen] {args.workload}: N={system.N:,} {system.counts()} in {time.perf_counter() - t0:.1f} s")

    # the timed window covers at least two Voronoi update periods, so the rate includes
    # the amortised cell updates, list builds and prunes
    steps = max(args.steps, 2 * mp.update_every)
    ctx, mixed = timed_run(R, mp, system, R.RBC_MIXED, steps, args.warmup, "mixed")
    list_bytes = list_output_bytes(ctx)
    n_ll, n_wca = pair_counts(ctx, system)
    n_bond = int(system.bonds.shape[0])
    ctx.close()
    flops = FLOPS_LIPID_PAIR * n_ll + FLOPS_WCA_PAIR * n_wca + FLOPS_BOND * n_bond
    n_lip = int(np.sum(system.type == 0))
    bytes_alg = BYTES_LIPID_STEP * n_lip + BYTES_PROTEIN_STEP * (system.N - n_lip)
    t_force = mixed["force_ms"] * 1e-3
    t_flop = flops / (PEAK_FP32 * 1e12)
    t_byte = bytes_alg / (PEAK_HBM * 1e9)
    if t_byte >= t_flop:
        bound, achieved, peak, unit = "hbm", bytes_alg / t_force / 1e9, PEAK_HBM, "GB/s"
    else:
        bound, achieved, peak, unit = "alu", flops / t_force / 1e12, PEAK_FP32, "TFLOP/s"
    digest = kernel_sources_digest()
    counters_valid = (FORCE_TRAFFIC["sources_sha256"] == digest and args.workload == "rbc4m" and
                      args.skin == FORCE_TRAFFIC["skin"] and args.inner_skin == FORCE_TRAFFIC["inner_skin"])
    traffic = FORCE_TRAFFIC["bytes"] if counters_valid else None
    # a wavefront VALU instruction occupies a 16-lane SIMD for 4 cycles
    valu_busy = (FORCE_TRAFFIC["valu_insts"] * 4 / (t_force * CLOCK_GHZ * 1e9 * CU_COUNT * SIMDS_PER_CU)
                 if counters_valid else None)
    roof = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel": "k_force<mixed, fused kick-drift-kick> (pair forces, bonds, integration)",
            "flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_alg,
            "pair_flops_tflops": round(flops / t_force / 1e12, 3),
            "pair_flops_frac_of_fp32_peak": round(flops / t_force / 1e12 / PEAK_FP32, 4),
            "avg_launch_us": round(mixed["force_ms"] * 1e3, 2), "launches_timed": mixed["force_launches"],
            "roofline_time_us": round(max(t_flop, t_byte) * 1e6, 2),
            "time_frac": round(max(t_flop, t_byte) / t_force, 4),
            "traffic_sources_sha256": digest,
            "hbm_traffic_tbps": round(traffic / t_force / 1e12, 3) if traffic else None,
            "valu_busy_frac": round(valu_busy, 4) if valu_busy else None,
            "lipid_pairs": n_ll, "wca_pairs": n_wca, "bonds": n_bond}
    log(f"[roofline] {roof}")
    build = build_roofline(mixed, list_bytes, system.N)
    log(f"[list build] {build}")

    fp64 = None
    if not args.no_fp64:
        ctx64, fp64 = timed_run(R, mp, system, R.RBC_FP64, args.fp64_steps, min(args.warmup, 10), "fp64")
        ctx64.close()
        fp64["force_tflops"] = flops / (fp64["force_ms"] * 1e-3) / 1e12
        fp64["force_frac_fp64_peak"] = fp64["force_tflops"] / PEAK_FP64

    ext = None
    if not args.no_ext:
        ext = ext_run(R, mp, system, args.detached_steps, min(args.warmup, 20))

    structure = None
    if not args.no_structure:
        structure = structure_run(R, mp, min(args.warmup, 20))

    detached = None
    if not args.no_detached:
        detached = detached_run(R, mp, args.workload, args.detached_steps, min(args.warmup, 20))

    configs = None
    if not args.no_configs:
        configs = {"patch_fp64": config_leg(R, mp, I.config("patch"), 100, 10, 100, "patch fp64"),
                   "vesicle_fp64": config_leg(R, mp, I.config("vesicle"), 1000, 10, 100, "vesicle fp64")}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(system, mp)
        log(f"[cpu] {cpu}")

    serving = None
    if not args.no_serving:
        smp = I.ModelParams(skin=args.skin, inner_skin=args.inner_skin)
        serving = serving_run(R, smp, args.serving_requests, 20.0, args.serving_steps)
        serving["saturated"] = serving_run(R, smp, args.serving_requests, 20.0, args.serving_steps, saturated=True)
        # the same arrivals with the step replayed as a HIP graph (direct launches are the default)
        g = serving_run(R, smp, args.serving_requests, 20.0, args.serving_steps, graphs=True)
        serving["graph_replay"] = {k: g[k] for k in ("step_latency_ms_p50", "step_latency_ms_p99",
                                                     "throughput_busy", "calls")}

    if args.calib_copy_mb > 0:
        nbytes = args.calib_copy_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[calib] copied {nbytes} bytes device to device")

    line = {
        "metric": "particle-steps/s at 4M-particle RBC; p50/p99 batched-ensemble step latency",
        "value": mixed["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic / f64 state",
        "data": "synthetic (seeded generator; no dataset)",
        "config": {"workload": f"{workload_shape(args.workload)} ({args.workload}), {system.N:,} particles: "
                               f"{system.counts()['L']:,} lipids, {system.counts()['J']:,} junctions, "
                               f"{system.counts()['S']:,} spectrin beads; dt={DT}, NVE, cells updated every "
                               f"{mp.update_every} steps, skin {mp.skin}, pruned-list buffer {mp.inner_skin}",
                   "particles": system.N, "precision": "mixed", "parallelism": "single GPU"},
        "roofline": roof,
        "list_build": build,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "mixed": mixed,
        "configs": configs,
        "serving": serving,
        "detached": detached,
        "volume_and_thermostat": ext,
        "structure": structure,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
