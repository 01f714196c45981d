#!/usr/bin/env python3
"""Benchmark of the batched collision step on one MI355X.

Workload: the batched collision step -- 4096 independent cells with
log-uniform particle counts in [64, 1024] (1.40e6 particles), log-uniform
masses 1e-12..1e2 g, random local gas, exactly 1000 collisions per cell per
step (seeded, synthetic).  A step is one mcd_step: every cell builds its rate
matrix row sums and performs its 1000 events (selection, outcome, rate
update); particles stay resident in HBM.

Reports collisions/s and algorithmic rate-pair evaluations/s for the four
forms {FP64, mixed} x {plain, batched}; the headline `value` is the mixed
batched form.  Adds the roofline of the collision kernel (vector-ALU bound),
the FP64 CPU oracle timed on a bounded sample of the same workload, and the
errors of the GPU forms against the oracle.

`full_step` times the whole path -- adaptive binning, collisions, transport --
on the large 2-D disk: 2e6 particles, 1000 x 10 equal-count cells of 200,
8 composition fractions, 1 yr per step with time-limited event loops, mixed
precision, graph-replayed steps; the binning alone is timed eagerly beside it.

`--copy-calibration` only runs an elementwise copy of 2^28 floats (1 GiB read,
1 GiB written) and exits: under `rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE`
it gives the factor between those counters and true HBM bytes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "collisions/sec + rate-pair evals/sec, mixed vs FP64 plain, at stated error"
# floating-point operations of one pair evaluation of the physical kernel,
# counted from the oracle's pair functions with per-particle and per-cell
# quantities precomputed (+ - * / sqrt = 1): Brownian 3, turbulence
# (intermediate regime) 14, drift and settling 9, sqrt 1, cross-section and
# kernel 4, two directed swarm rates with grouping 2 x 4
F_PAIR = 39
PEAK_FP32_TFLOPS = 157.3
EVENTS_PER_CELL = 1000

# HBM traffic of one launch of the collision kernel on this workload, from
# `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs (KiB per dispatch),
# scaled by the same counters' reading for an elementwise copy of known size
# (a 1 GiB read shows as 524288 KiB of FETCH_SIZE, a 1 GiB write as 1048576 KiB
# of WRITE_SIZE: factors 2.0 and 1.0).
# Valid only for the kernel sources it was taken on: their SHA-256 is kept
# and compared at run time; on any change `traffic` is reported as null.
TRAFFIC = {"fetch_kib": 17094.75, "write_kib": 24237.38, "fetch_factor": 1.99994, "write_factor": 1.0,
           "sources_sha256": "b456778d1a29b4d439a31df0de2e3d5e3b98253a59169af6acf78d0de26737f0"}
# Issue rate of the same launch from one `rocprofv3 --pmc` pass of SQ counters:
# VALU busy = 4 * SQ_ACTIVE_INST_VALU / (1024 SIMDs * launch cycles at 2.4 GHz),
# and SQ_INSTS_VALU per collision; the same validity rule as TRAFFIC.
ISSUE = {"valu_busy": 0.843, "valu_insts_per_collision": 1615,
         "sources_sha256": "b456778d1a29b4d439a31df0de2e3d5e3b98253a59169af6acf78d0de26737f0"}
KERNEL_SOURCES = ("paper_2507_21239_amd/csrc/collide.hip", "paper_2507_21239_amd/csrc/collide_device.hpp",
                  "paper_2507_21239_amd/csrc/collide_ilp.hip", "paper_2507_21239_amd/csrc/physics.hpp",
                  "paper_2507_21239_amd/csrc/device_common.hpp", "paper_2507_21239_amd/csrc/internal.hpp",
                  "paper_2507_21239_amd/build.py")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes():
    """Counter-derived HBM bytes per launch, or None if the kernel changed."""
    t = TRAFFIC
    if t["fetch_kib"] is None or t["sources_sha256"] != kernel_sources_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])


def issue_rate():
    """Counter-derived VALU busy fraction and instructions per collision, or
    (None, None) if the kernel changed."""
    if ISSUE["sources_sha256"] != kernel_sources_sha256():
        return None, None
    return ISSUE["valu_busy"], ISSUE["valu_insts_per_collision"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pair_evals(counts, events):
    counts = counts.astype("float64")
    return float((counts * (counts + 1) / 2).sum() + events * counts.sum())


def executed_pair_evals(counts, events, small_max=256):
    """Pair evaluations the mixed batched kernel executes, lane by lane
    (padded slots included): cells up to small_max on one wave (K = ceil(n/64)
    slots per lane), larger ones on four-wave teams (K = ceil(n/256)).  The
    pairwise FP32 build evaluates per lane the K(K+1)/2 pairs of its own
    slots, then K^2 pairs at each of 32 lane offsets of its own wave and, in
    four-wave teams, at 3 x 32 offsets of the other waves; every event
    evaluates each slot twice (row i before and after the outcome)."""
    import numpy as np
    n = counts.astype("int64")
    one = n <= small_max
    lanes = np.where(one, 64, 256)
    K = np.where(one, (n + 63) // 64, (n + 255) // 256)
    offsets = np.where(one, 32, 32 + 3 * 32)
    build = lanes * (K * (K + 1) // 2 + offsets * K * K)
    passes = events * 2 * lanes * K
    return float((build + passes).sum())


FIXED_SCHEDULE = None   # (small_max, grid_per_cu) from --schedule


def choose_schedule(sim, dt, max_events):
    if FIXED_SCHEDULE is not None:
        sim.set_schedule(*FIXED_SCHEDULE)
        return {"small_max": FIXED_SCHEDULE[0], "grid_per_cu": FIXED_SCHEDULE[1], "fixed": True}
    return sim.tune(dt, max_events)


def run_mode(work, precision, schedule, steps, warmup):
    """Plain: one workgroup per cell, each step launched by itself, no
    tuning.  Batched: persistent launch, autotuned schedule, the K timed steps
    replayed from a captured HIP graph (captured during the warm-up)."""
    import numpy as np
    import torch
    from paper_2507_21239_amd import api
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision=precision, schedule=schedule)
    # the workload's largest cell bounds the cells: planned on the device, no sync
    sim.bin(api.cells_to_device(work["cells"]), max_cell=int(np.diff(work["cells"]["cell_start"]).max()))
    tuned = None
    if schedule == "batched":
        tuned = choose_schedule(sim, 0.0, EVENTS_PER_CELL)
        if warmup >= 2:
            sim.step(0.0, EVENTS_PER_CELL, warmup)
        elif warmup == 1:
            sim.step(0.0, EVENTS_PER_CELL, 1)
    else:
        for _ in range(warmup):
            sim.step(0.0, EVENTS_PER_CELL, 1)
    torch.cuda.synchronize()
    ev0 = sim.stats()["events"]
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(stream)
    if schedule == "batched":
        sim.step(0.0, EVENTS_PER_CELL, steps)
    else:
        for _ in range(steps):
            sim.step(0.0, EVENTS_PER_CELL, 1)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = sim.stats()
    sim.close()
    kernel_ms = a.elapsed_time(b) / steps
    return dict(wall_s=wall, ms_per_step=wall / steps * 1e3, kernel_ms=kernel_ms,
                events=st["events"] - ev0, schedule=tuned)


def full_step(steps, warmup, steady=True):
    """Whole path on the large 2-D disk: bin -> collide -> transport per step;
    an early window (after the warm-up), a late one (steps LATE_FROM ..) and,
    with steady, the steady state (steps STEADY_FROM ..)."""
    import numpy as np
    import torch
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W
    work = W.c5_large_disk(seed=0)
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
    stream = torch.cuda.current_stream()
    sim.bin()
    tuned = choose_schedule(sim, W.YR, 0)
    if warmup > 0:
        sim.step(W.YR, 0, warmup)   # with warmup >= 2 this also captures the step graph
    torch.cuda.synchronize()
    # binning alone, eager, on the state the timed steps start from
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        sim.bin()
    b.record(stream)
    torch.cuda.synchronize()
    bin_ms = a.elapsed_time(b) / steps
    ev0 = sim.stats()["events"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(stream)
    sim.step(W.YR, 0, steps)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_main = a.elapsed_time(b) / steps
    st = sim.stats()
    events = st["events"] - ev0
    # a late window: the busiest cells' event chains grow with the disk's
    # age, and with them the step (steps LATE_FROM .. LATE_FROM + LATE_STEPS - 1)
    done = warmup + steps
    if done < LATE_FROM:
        sim.step(W.YR, 0, LATE_FROM - done)
    ev1 = sim.stats()["events"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a.record(stream)
    sim.step(W.YR, 0, LATE_STEPS)   # graph replays, as in the main window
    b.record(stream)
    torch.cuda.synchronize()
    wall_late = time.perf_counter() - t1
    gpu_late = a.elapsed_time(b) / LATE_STEPS
    late_events = sim.stats()["events"] - ev1
    n = len(work["particles"]["m"])
    out = {"workload": "2-D disk 1-100 AU: 2e6 particles, 1000 x 10 equal-count cells of 200, "
                       "8 composition fractions, drift + settling + mixing + coagulation, "
                       "1 yr per step, time-limited events",
           "precision": "mixed", "schedule": "batched", "steps": steps, "warmup": warmup,
           "particles": n, "active": int(st["n_active"]),
           "ms_per_step": wall / steps * 1e3, "gpu_ms_per_step": gpu_main,
           "events_per_step": events / steps, "collisions_per_s": events / wall,
           "bin_ms": bin_ms, "tuned_schedule": tuned,
           "late_window": {"from_step": max(LATE_FROM, done), "steps": LATE_STEPS,
                           "ms_per_step": wall_late / LATE_STEPS * 1e3,
                           "gpu_ms_per_step": gpu_late,
                           "events_per_step": late_events / LATE_STEPS,
                           "collisions_per_s": late_events / wall_late}}
    if steady:
        # the disk in its steady state (steps STEADY_FROM ..): time a window,
        # then count one step's events per cell with the event log (the
        # busiest cells' serial chains bound the collision launch from below)
        at = max(LATE_FROM, done) + LATE_STEPS
        if at < STEADY_FROM:
            sim.step(W.YR, 0, STEADY_FROM - at)
        ev2 = sim.stats()["events"]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        a.record(stream)
        sim.step(W.YR, 0, STEADY_STEPS)
        b.record(stream)
        torch.cuda.synchronize()
        wall_steady = time.perf_counter() - t2
        gpu_steady = a.elapsed_time(b) / STEADY_STEPS
        steady_events = sim.stats()["events"] - ev2
        # the same state under other fixed schedules (10 steps each): more or
        # fewer workgroups per CU, and four-wave teams for the 200-particle cells
        by_schedule = {}
        for sm, g in ((256, 1), (256, 3), (128, 2)):
            sim.set_schedule(sm, g)
            sim.step(W.YR, 0, 1)
            torch.cuda.synchronize()
            a.record(stream)
            sim.step(W.YR, 0, 10)
            b.record(stream)
            torch.cuda.synchronize()
            by_schedule[f"{sm},{g}"] = a.elapsed_time(b) / 10
        if tuned and "small_max" in tuned:
            sim.set_schedule(tuned["small_max"], tuned["grid_per_cu"])
        n_cells = len(sim.cells()["cell_start"]) - 1
        per = 4096
        log_buf = torch.full((n_cells * per * 4,), -2, dtype=torch.int32, device="cuda")
        sim.set_event_log(log_buf, per)
        sim.step(W.YR, 0, 1)
        sim.set_event_log(None)
        torch.cuda.synchronize()
        per_cell = (log_buf.view(n_cells, per, 4)[:, :, 0] != -2).sum(dim=1).cpu().numpy()
        del log_buf
        out["steady_window"] = {
            "from_step": max(STEADY_FROM, at), "steps": STEADY_STEPS,
            "ms_per_step": wall_steady / STEADY_STEPS * 1e3,
            "gpu_ms_per_step": gpu_steady,
            "gpu_ms_per_step_by_schedule_after": by_schedule,
            "events_per_step": steady_events / STEADY_STEPS,
            "collisions_per_s": steady_events / wall_steady,
            "events_per_cell_one_step": {
                "max": int(per_cell.max()), "p99": float(np.percentile(per_cell, 99)),
                "p90": float(np.percentile(per_cell, 90)), "median": float(np.median(per_cell)),
                "cells_at_log_cap": int((per_cell >= per).sum())}}
    sim.close()
    return out


def steady_state(steps):
    """The large disk in its steady state alone, for profiling: STEADY_FROM
    untimed steps (schedule tuned on the initial state, or fixed by
    --schedule), then `steps` timed steps; in a kernel trace the last `steps`
    launches of each kernel are the steady ones."""
    import torch
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W
    work = W.c5_large_disk(seed=0)
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
    sim.bin()
    tuned = choose_schedule(sim, W.YR, 0)
    done = 0
    while done < STEADY_FROM:
        k = min(100, STEADY_FROM - done)
        sim.step(W.YR, 0, k)
        done += k
        torch.cuda.synchronize()
        log("steady state:", done, "steps")
    ev0 = sim.stats()["events"]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    sim.step(W.YR, 0, steps)
    b.record()
    torch.cuda.synchronize()
    ev = sim.stats()["events"] - ev0
    sim.close()
    return {"from_step": STEADY_FROM, "steps": steps, "gpu_ms_per_step": a.elapsed_time(b) / steps,
            "events_per_step": ev / steps, "tuned_schedule": tuned}


LATE_FROM, LATE_STEPS = 20, 20
STEADY_FROM, STEADY_STEPS = 300, 20
CLOCK_GHZ = 2.4


def _lone_sim(n, small_max, n_comp, events, grid_per_cu):
    """A Simulation holding one cell of n particles (the batched workload's
    particle recipe), n_comp one-hot composition fractions, mixed, batched."""
    import numpy as np
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W
    work = W.c4_batched(seed=9, counts=[n], events=events)
    if n_comp:
        work["params"] = dict(work["params"], n_comp=n_comp)
        comp = np.zeros((n_comp, n), dtype=np.float32)
        comp[np.arange(n) % n_comp, np.arange(n)] = 1.0
        work["particles"]["comp"] = comp
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
    sim.bin(api.cells_to_device(work["cells"]), max_cell=n)
    sim.set_schedule(small_max, grid_per_cu)
    return sim


def lone_counting(spec, events, launches):
    """One cell alone for instruction counters: spec "N" or "N,n_comp" (one
    wave up to 256 particles, a four-wave team above), `launches` collision
    launches of `events` events each after one warm-up launch, one workgroup
    per CU (fewer idle waves in the counters).  Two runs that differ only in
    `events` give the counts per event as the difference."""
    import torch
    parts = [int(x) for x in spec.split(",")]
    n, n_comp = parts[0], (parts[1] if len(parts) > 1 else 0)
    sim = _lone_sim(n, 256, n_comp, events, 1)
    sim.step(0.0, events, 1)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    sim.step(0.0, events, launches)
    b.record()
    torch.cuda.synchronize()
    out = {"particles": n, "n_comp": n_comp, "events_per_launch": events, "launches": launches,
           "us_per_launch": a.elapsed_time(b) * 1e3 / launches,
           "events_total": int(sim.stats()["events"])}
    sim.close()
    return out


def lone_cells():
    """Latency of one cell's serial event chain: a single cell alone on the
    GPU (mixed, batched schedule: one wave up to 256 particles, a four-wave
    team above), 1000 events, HIP events around the launch after one
    warm-up step; cycles at the 2.4 GHz peak clock.  Also a 200-particle cell
    on a four-wave team (single-wave threshold 199) and one carrying 8
    composition fractions (the kernel variant with the composition mix)."""
    import torch
    out = {}
    for name, n, small_max, n_comp in (("64", 64, 256, 0), ("200", 200, 256, 0),
                                       ("256", 256, 256, 0), ("1000", 1000, 256, 0),
                                       ("200_four_wave", 200, 199, 0), ("200_comp8", 200, 256, 8)):
        sim = _lone_sim(n, small_max, n_comp, EVENTS_PER_CELL, 0)
        sim.step(0.0, EVENTS_PER_CELL, 1)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        sim.step(0.0, EVENTS_PER_CELL, 1)
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / EVENTS_PER_CELL
        sim.close()
        out[name] = {"particles": n, "waves": 1 if n <= small_max else 4, "n_comp": n_comp,
                     "us_per_event": us, "cycles_per_event": us * 1e-6 * CLOCK_GHZ * 1e9}
    return out


def next_rows(steps, warmup):
    """Cost of the features beyond the collision step, measured on the
    workloads they serve (mixed, batched, fixed schedule 256,0 so that no
    tuning trials enter the timings):
    - the large disk's whole step with the power-law gas and with a gridded gas
      (48 x 24 nodes; the gas is sampled per cell, per particle in transport and
      once per cell for eta v_K);
    - the batched workload's collision step with the sharp fragmentation
      criterion and with the ramp and Maxwell criteria (their kernel variant);
    - the large disk's step with an asynchronous snapshot of (r, z, m, active,
      comp) after every step, against none;
    - one sigma_d(m, r) histogram of the large disk, 60 radial x 64 mass bins."""
    import numpy as np
    import torch
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W

    def timed(sim, run):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, a.elapsed_time(b)

    def disk(gas_grid=None, snapshot=False):
        work = W.c5_large_disk(seed=0)
        dev = api.to_device(work["particles"])
        sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
        if gas_grid is not None:
            sim.set_gas_grid(gas_grid)
        sim.bin()
        sim.set_schedule(256, 0)
        sim.step(W.YR, 0, max(warmup, 2))
        bufs, snaps = [], []
        if snapshot:
            # a first snapshot sizes the library's staging; then two rotating pinned buffers
            first = sim.snapshot()
            first.wait()
            bufs = [torch.empty_like(first.buf, pin_memory=True) for _ in range(2)]

        def run():
            if not snapshot:
                sim.step(W.YR, 0, steps)
                return
            for k in range(steps):
                sim.step(W.YR, 0, 1)
                if len(snaps) == 2:
                    snaps.pop(0).wait()
                snaps.append(sim.snapshot(out=bufs[k % 2]))
            for sn in snaps:
                sn.wait()
        wall, gpu = timed(sim, run)
        sim.close()
        return {"ms_per_step": wall / steps, "gpu_ms_per_step": gpu / steps}

    def c4(frag_mode):
        work = W.c4_batched(seed=0, events=EVENTS_PER_CELL)
        p = dict(work["params"])
        p["frag_mode"] = frag_mode
        dev = api.to_device(work["particles"])
        sim = api.Simulation(p, dev, precision="mixed", schedule="batched")
        sim.bin(api.cells_to_device(work["cells"]))
        sim.set_schedule(256, 0)
        sim.step(0.0, EVENTS_PER_CELL, max(warmup, 2))
        wall, gpu = timed(sim, lambda: sim.step(0.0, EVENTS_PER_CELL, steps))
        out = sim.stats()["outcomes"]
        sim.close()
        return {"ms_per_step": wall / steps, "outcomes_since_init": [int(x) for x in out]}

    res = {}
    log("next rows: large disk, power-law gas")
    res["disk_power_law"] = disk()
    log("next rows: large disk, gridded gas")
    res["disk_gridded_gas"] = disk(gas_grid=W.gridded_gas(W.c5_large_disk(seed=0)["params"]))
    log("next rows: large disk, snapshot after every step")
    res["disk_snapshot_every_step"] = disk(snapshot=True)
    for mode in ("sharp", "ramp", "maxwell"):
        log("next rows: batched workload, fragmentation", mode)
        res[f"c4_frag_{mode}"] = c4(mode)
    log("next rows: sigma_d histogram")
    work = W.c5_large_disk(seed=0)
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
    re = W.AU * np.logspace(0.0, 2.0, 61)
    me = np.logspace(-14.0, 4.0, 65)
    sim.sigma_hist(re, me)
    reps = 10
    wall, gpu = timed(sim, lambda: [sim.sigma_hist(re, me) for _ in range(reps)])
    sim.close()
    res["sigma_hist_60x64"] = {"ms": gpu / reps, "particles": len(work["particles"]["m"])}
    return res


def configs_table(steps=10):
    """Per-configuration rates of the GPU forms and of the FP64 oracle, on the
    parity-test configurations (one cell with the constant kernel; one column;
    the 1e5-particle disk) and the 2e6-particle disk.  GPU: FP64 plain and
    mixed batched (autotuned), `steps` steps after 2 warm-ups (the single
    cell: its one step to t = 1998, three fresh runs); oracle: every host core,
    the first steps of the same run.  Collisions/s = events / wall time of
    the steps (binning and transport included where the configuration has
    them)."""
    import numpy as np
    import torch

    import oracle as O
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W

    threads = host_threads()

    def fresh(work):
        return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in work["particles"].items()}

    def gpu(work, precision, schedule, n):
        dev = api.to_device(fresh(work))
        sim = api.Simulation(work["params"], dev, precision=precision, schedule=schedule)
        sim.bin(api.cells_to_device(work["cells"]) if work["cells"] is not None else None)
        dt, me = work["dt"], work.get("max_events", 0)
        if schedule == "batched":
            choose_schedule(sim, dt, me)
        if n > 1:
            sim.step(dt, me, 2)
        ev0 = sim.stats()["events"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(dt, me, n)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev = sim.stats()["events"] - ev0
        sim.close()
        return wall, ev

    def oracle(work, n):
        part = fresh(work)
        t0 = time.perf_counter()
        ev = 0
        for s in range(n):
            out = O.step(work["params"], part, s, work["dt"], work.get("max_events", 0),
                         cells=work["cells"], threads=threads)
            ev += int(out["stats"]["events"].sum())
        return time.perf_counter() - t0, ev

    def row(name, work, g_steps, o_steps, reps=1):
        r = {"particles": len(work["particles"]["m"])}
        for precision, schedule in (("fp64", "plain"), ("mixed", "batched")):
            log("configs:", name, precision, schedule)
            runs = [gpu(work, precision, schedule, g_steps) for _ in range(reps)]
            wall, ev = sorted(runs)[len(runs) // 2]
            r[f"gpu_{precision}_{schedule}"] = {"ms_per_step": wall / g_steps * 1e3,
                                                "events_per_step": ev / g_steps,
                                                "collisions_per_s": ev / wall}
        log("configs:", name, "oracle")
        runs = [oracle(work, o_steps) for _ in range(reps)]
        wall, ev = sorted(runs)[len(runs) // 2]
        r["oracle"] = {"threads": threads, "steps": o_steps, "ms_per_step": wall / o_steps * 1e3,
                       "events_per_step": ev / o_steps, "collisions_per_s": ev / wall}
        return r

    res = {}
    res["single_cell_constant_kernel"] = row("single cell", W.c1_single_cell(seed=0), 1, 1, reps=3)
    res["column_20x200"] = row("column", W.c2_column(seed=0), steps, 20)
    res["disk_1e5"] = row("disk 1e5", W.c3_disk(seed=0), steps, 10)
    res["disk_2e6"] = row("disk 2e6", W.c5_large_disk(seed=0), steps, 1)
    return res


def copy_calibration():
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    log("copy calibration: 1 elementwise kernel, 1073741824 B read, 1073741824 B written")


def error_report(work, n_sample=8):
    """Errors of the GPU forms against the FP64 oracle on sampled cells."""
    import ctypes as C

    import numpy as np
    import torch

    import oracle as O
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W

    cs = work["cells"]["cell_start"]
    sizes = np.diff(cs)
    rng = np.random.default_rng(123)
    pick = sorted(set([int(np.argmax(sizes))] + list(rng.choice(len(sizes), n_sample - 1, replace=False))))
    out = {"sample_cells": len(pick)}
    # rate matrices
    worst = {}
    for precision in ("fp64", "mixed"):
        dev = api.to_device(work["particles"])
        sim = api.Simulation(work["params"], dev, precision=precision)
        sim.bin(api.cells_to_device(work["cells"]))
        w = 0.0
        for c in pick:
            n = int(sizes[c])
            Rg, _ = sim.rates(c, n)
            Ro, _ = O.cell_rates(work["params"], work["cells"]["gas"][c],
                                 work["cells"]["order"][cs[c]:cs[c + 1]],
                                 work["particles"]["m"], work["particles"]["M"])
            w = max(w, float(np.max(np.abs(Rg.cpu().numpy() - Ro) / Ro)))
        worst[precision] = w
        sim.close()
    out["rate_max_rel_err_fp64"] = worst["fp64"]
    out["rate_max_rel_err_mixed"] = worst["mixed"]
    # one step: FP64 event sequences and final masses of sampled cells
    logs = {}
    masses = {}
    for precision in ("fp64", "mixed"):
        dev = api.to_device(work["particles"])
        sim = api.Simulation(work["params"], dev, precision=precision)
        sim.bin(api.cells_to_device(work["cells"]))
        buf = torch.full((len(sizes) * EVENTS_PER_CELL * 4,), -7, dtype=torch.int32, device="cuda")
        sim.set_event_log(buf, EVENTS_PER_CELL)
        sim.step(0.0, EVENTS_PER_CELL, 1)
        logs[precision] = buf.cpu().numpy().reshape(len(sizes), EVENTS_PER_CELL, 4)
        masses[precision] = dev["m"].cpu().numpy()
        sim.close()
    mism, mrel = 0, 0.0
    om_all, gm_all = [], []
    for c in pick:
        sub = W.subset_cells(work, np.array([c]))
        part = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sub["particles"].items()}
        lg = np.zeros(EVENTS_PER_CELL, dtype=O.EVENT_DTYPE)
        st = np.zeros(1, dtype=O.STATS_DTYPE)
        O.lib().orc_collide_cell(C.byref(O.make_params(sub["params"])),
                                 O._ptr(np.ascontiguousarray(sub["cells"]["gas"][0]), C.c_double),
                                 c, 0, int(sizes[c]),
                                 O._ptr(np.ascontiguousarray(sub["cells"]["order"]), C.c_int32),
                                 O._ptr(part["m"], C.c_double), O._ptr(part["M"], C.c_double),
                                 None, len(part["m"]), 0.0, EVENTS_PER_CELL, lg.ctypes.data,
                                 EVENTS_PER_CELL, st.ctypes.data)
        o = np.stack([lg["i"], lg["j"], lg["outcome"]], axis=1)
        mism += int(np.any(o != logs["fp64"][c, :, :3], axis=1).sum())
        g = masses["fp64"][cs[c]:cs[c + 1]]
        mrel = max(mrel, float(np.max(np.abs(g - part["m"]) / part["m"])))
        om_all.append(np.log10(part["m"]))
        gm_all.append(np.log10(masses["mixed"][cs[c]:cs[c + 1]]))
    out["fp64_event_mismatches"] = mism
    out["fp64_events_compared"] = len(pick) * EVENTS_PER_CELL
    out["fp64_mass_max_rel_err"] = mrel
    from scipy import stats as sst
    # paired: the same cells on the same Philox stream, so the two forms mostly
    # take the same events; a distance, not a test (the ensembles below are)
    ks = sst.ks_2samp(np.concatenate(om_all), np.concatenate(gm_all))
    out["mixed_vs_oracle_same_stream_logm_ks_D"] = float(ks.statistic)
    return out


def swarm_summary(m, M, active):
    """Per-run summary of the active swarms (M_k = sum N_i m_i^k, N_i = M_i/m_i):
    the moment ratios M1/M0, M2/M1, M3/M2, the mass-weighted mean log10 m and
    the active count."""
    import numpy as np
    a = np.asarray(active).astype(bool)
    m, M = np.asarray(m)[a], np.asarray(M)[a]
    N = M / m
    return {"M1/M0": M.sum() / N.sum(), "M2/M1": (M * m).sum() / M.sum(),
            "M3/M2": (M * m * m).sum() / (M * m).sum(),
            "mass-weighted mean log10 m": float((M * np.log10(m)).sum() / M.sum()),
            "active": float(a.sum())}


def compare_ensembles(a_runs, b_runs, a_name, b_name):
    """Two ensembles of independent runs (disjoint seeds): per quantity the
    means, standard errors over seeds and the difference in units of its
    standard error (z); two-sample KS on the pooled log10 m of the
    representative particles (they sample the mass distribution).  The
    particles of one run are not independent of each other, so the KS
    distance is judged against a permutation of whole runs between the two
    sides (p_runs_permutation); the particle-level p-value and the distance
    between the two halves of each ensemble are reported beside it.
    Tolerances: |z| <= 3 for every quantity and a permutation p above 0.01."""
    import numpy as np
    from scipy import stats as sst
    out = {"runs": {a_name: len(a_runs), b_name: len(b_runs)}, "quantities": {}}
    ok = True
    for q in a_runs[0]["summary"]:
        xa = np.array([r["summary"][q] for r in a_runs])
        xb = np.array([r["summary"][q] for r in b_runs])
        sa, sb = xa.std(ddof=1) / np.sqrt(len(xa)), xb.std(ddof=1) / np.sqrt(len(xb))
        se = float(np.hypot(sa, sb))
        z = float((xb.mean() - xa.mean()) / se) if se > 0 else (0.0 if xb.mean() == xa.mean() else float("inf"))
        ok = ok and abs(z) <= 3.0
        out["quantities"][q] = {a_name: float(xa.mean()), a_name + "_se": float(sa),
                                b_name: float(xb.mean()), b_name + "_se": float(sb), "z": z}
    la = [r["logm"] for r in a_runs]
    lb = [r["logm"] for r in b_runs]
    ks = sst.ks_2samp(np.concatenate(la), np.concatenate(lb))
    h = lambda L: sst.ks_2samp(np.concatenate(L[: len(L) // 2]), np.concatenate(L[len(L) // 2:])).statistic
    ref = max(float(h(la)), float(h(lb)))
    # the run-permutation reference, on 1e-4 dex histograms of the runs
    p_perm = _ks_permutation_p([_logm_hist(x) for x in la], [_logm_hist(x) for x in lb])
    out["logm_ks"] = {"D": float(ks.statistic), "p_particles": float(ks.pvalue),
                      "p_runs_permutation": p_perm, "D_half_vs_half": ref,
                      "samples": [int(sum(map(len, la))), int(sum(map(len, lb)))]}
    ok = ok and p_perm > 0.01
    out["within_tolerance"] = bool(ok)
    return out


def _gpu_disk_run(work_fn, seed, precision, steps, tune=True):
    import numpy as np
    import torch
    from paper_2507_21239_amd import api
    from paper_2507_21239_amd import workloads as W
    work = work_fn(seed)
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision=precision, schedule="batched")
    sim.bin()
    if tune:
        choose_schedule(sim, W.YR, 0)
    done = 0
    while done < steps:   # chunks, so that a long run reports its progress
        k = min(2000, steps - done)
        sim.step(W.YR, 0, k)
        done += k
        if done < steps:
            torch.cuda.synchronize()
            log("  ", precision, "seed", seed, done, "steps")
    ev = sim.stats()["events"]
    torch.cuda.synchronize()
    h = {k: dev[k].cpu().numpy() for k in ("m", "active")}
    sim.close()
    act = h["active"].astype(bool)
    return {"summary": swarm_summary(h["m"], work["particles"]["M"], act),
            "logm": np.log10(h["m"][act]), "events": int(ev)}


def _oracle_disk_run(work_fn, seed, steps):
    import numpy as np
    import oracle as O
    work = work_fn(seed)
    part = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in work["particles"].items()}
    ev = 0
    for s in range(steps):
        ev += int(O.step(work["params"], part, s, work["dt"], 0,
                         threads=host_threads())["stats"]["events"].sum())
    act = part["active"].astype(bool)
    return {"summary": swarm_summary(part["m"], part["M"], act), "logm": np.log10(part["m"][act]),
            "events": ev}


def ensemble_report(seeds=16, steps=40):
    """The mixed GPU form against the FP64 oracle as independent ensembles:
    the Benchmark table's disk with 1e5 particles in 50 x 10 cells (drift,
    settling, mixing, coagulation, 1 yr per step), `steps` steps from the
    same initial state; the oracle with Philox seeds 0..seeds-1, the mixed
    form with seeds seeds..2 seeds-1.  The two ensembles share no random
    numbers, so their difference is a distributional one."""
    from paper_2507_21239_amd import workloads as W
    fn = lambda seed: dict(W.c3_disk(seed=0), params=dict(W.c3_disk(seed=0)["params"], seed=seed))
    t0 = time.perf_counter()
    orc = [_oracle_disk_run(fn, s, steps) for s in range(seeds)]
    t1 = time.perf_counter()
    mix = [_gpu_disk_run(fn, seeds + s, "mixed", steps) for s in range(seeds)]
    out = compare_ensembles(orc, mix, "oracle", "mixed")
    out.update({"workload": "2-D disk 1-100 AU, 1e5 particles, 50 x 10 cells, 1 yr per step",
                "horizon_yr": steps, "oracle_seeds": [0, seeds - 1],
                "mixed_seeds": [seeds, 2 * seeds - 1], "oracle_s": t1 - t0,
                "events_per_run": {"oracle": float(sum(r["events"] for r in orc) / seeds),
                                   "mixed": float(sum(r["events"] for r in mix) / seeds)}})
    return out


def large_disk_ensemble(seeds=16, years=1000, oracle_steps=3):
    """The large disk (2e6 particles, 1000 x 10 cells, 8 composition
    fractions) as 16-seed ensembles: the mixed form (seeds 16..31) against
    GPU FP64 (seeds 0..15) over `years` steps of 1 yr (none if years is 0) -- GPU FP64 stands in
    for the oracle at this size and horizon (it takes the oracle's event
    decisions bit for bit on short horizons) -- and against the oracle
    itself (seeds 0..15) over the first `oracle_steps` steps."""
    from paper_2507_21239_amd import workloads as W
    fn = lambda seed: dict(W.c5_large_disk(seed=0), params=dict(W.c5_large_disk(seed=0)["params"], seed=seed))
    res = {"workload": "2-D disk 1-100 AU, 2e6 particles, 1000 x 10 cells of 200, 8 composition "
                       "fractions, 1 yr per step"}
    t0 = time.perf_counter()
    f64, mix = [], []
    if years > 0:
        log("ensemble: large disk, FP64 GPU seeds 0..", seeds - 1, years, "yr")
        for s in range(seeds):
            f64.append(_gpu_disk_run(fn, s, "fp64", years))
            log("ensemble: fp64 seed", s, "done,", f"{time.perf_counter() - t0:.1f} s")
        t_mid = time.perf_counter()
        for s in range(seeds):
            mix.append(_gpu_disk_run(fn, seeds + s, "mixed", years))
            log("ensemble: mixed seed", seeds + s, "done,", f"{time.perf_counter() - t0:.1f} s")
        res["mixed_vs_gpu_fp64"] = dict(compare_ensembles(f64, mix, "fp64", "mixed"),
                                        horizon_yr=years, fp64_s_per_run=(t_mid - t0) / seeds,
                                        mixed_s_per_run=(time.perf_counter() - t_mid) / seeds)
    log("ensemble: large disk, oracle", oracle_steps, "steps")
    t1 = time.perf_counter()
    orc = []
    for s in range(seeds):
        orc.append(_oracle_disk_run(fn, s, oracle_steps))
        log("ensemble: oracle seed", s, "done,", f"{time.perf_counter() - t1:.1f} s")
    t2 = time.perf_counter()
    mix_s = [_gpu_disk_run(fn, seeds + s, "mixed", oracle_steps, tune=False) for s in range(seeds)]
    res["mixed_vs_oracle"] = dict(compare_ensembles(orc, mix_s, "oracle", "mixed"),
                                  horizon_yr=oracle_steps, oracle_s=t2 - t1)
    return res


LOGM_EDGES = (-16.0, 8.0, 240_000)   # log10 m histogram of a run: 1e-4 dex bins


def _logm_hist(logm):
    import numpy as np
    lo, hi, nb = LOGM_EDGES
    return np.histogram(np.clip(logm, lo, hi - 1e-9), bins=nb, range=(lo, hi))[0].astype(np.int64)


def _ks_permutation_p(hists_a, hists_b, n_perm=1000):
    """Permutation p-value of the pooled KS distance between two ensembles of
    runs: the runs are exchangeable if both sides sample the same
    distribution, so the run labels are shuffled (n_perm times, fixed seed)
    and the pooled distance recomputed; p = share of shuffles at least as far
    apart as observed.  Whole runs move together, so the run-to-run spread
    (not only the particle count) sets the reference."""
    import numpy as np
    H = np.stack(list(hists_a) + list(hists_b)).astype(np.float64)
    # 1e-2 dex for the reference distribution (the observed distance on the
    # same grid), so that a thousand shuffles take a second
    H = H.reshape(len(H), -1, 100).sum(axis=2)
    C = np.cumsum(H, axis=1)
    na, n = len(hists_a), len(H)

    def dist(sel):
        ca, cb = sel @ C, (1.0 - sel) @ C
        return np.max(np.abs(ca / ca[:, -1:] - cb / cb[:, -1:]), axis=1)

    obs = np.zeros((1, n))
    obs[0, :na] = 1.0
    d0 = float(dist(obs)[0])
    rng = np.random.default_rng(12345)
    sel = np.zeros((n_perm, n))
    for k in range(n_perm):
        sel[k, rng.permutation(n)[:na]] = 1.0
    return float((np.sum(dist(sel) >= d0) + 1) / (n_perm + 1))


def large_disk_ensemble_part(first, count, years, out_path, seeds=16, sides=("fp64", "mixed"),
                             same_seeds=False):
    """Runs first .. first+count-1 of the large disk's 16-seed ensembles over
    `years` steps of 1 yr, for each of `sides`: GPU FP64 with seed s, the
    oracle with seed s (on the host CPU only), mixed with seed 16 + s; saved to
    out_path (per run: the summary, the event count, the wall time and a
    histogram of log10 m of the active particles), so that a horizon too long
    for one sitting can be run in parts, and the oracle apart from the GPU,
    and combined with large_disk_ensemble_combine.  same_seeds: the mixed runs
    take seed s too (shared Philox streams, for a paired comparison)."""
    import numpy as np
    from paper_2507_21239_amd import workloads as W
    fn = lambda seed: dict(W.c5_large_disk(seed=0), params=dict(W.c5_large_disk(seed=0)["params"], seed=seed))
    rec = {}
    for s in range(first, first + count):
        for side in sides:
            seed = seeds + s if side == "mixed" and not same_seeds else s
            t0 = time.perf_counter()
            r = _oracle_disk_run(fn, seed, years) if side == "oracle" else \
                _gpu_disk_run(fn, seed, side, years)
            wall = time.perf_counter() - t0
            log("ensemble part:", side, "seed", seed, f"{wall:.1f} s")
            key = f"{side}_{seed}"
            rec[key + "_summary"] = np.array([r["summary"][q] for q in SUMMARY_KEYS])
            rec[key + "_events"] = np.array(r["events"])
            rec[key + "_wall"] = np.array(wall)
            rec[key + "_hist"] = _logm_hist(r["logm"])
    np.savez_compressed(out_path, years=np.array(years), **rec)
    return {"saved": out_path, "runs": len(rec) // 4}


SUMMARY_KEYS = ("M1/M0", "M2/M1", "M3/M2", "mass-weighted mean log10 m", "active")


def compare_ensembles_hist(a_runs, b_runs, a_name, b_name):
    """compare_ensembles for runs that carry a histogram of log10 m (1e-4 dex
    bins) instead of the samples: the KS distance is the largest gap of the
    pooled empirical distribution functions at the bin edges (exact up to
    the mass of one bin), its particle-level p-value from the asymptotic
    Kolmogorov law, and the same run-permutation reference and tolerances."""
    import numpy as np
    from scipy import special
    out = {"runs": {a_name: len(a_runs), b_name: len(b_runs)}, "quantities": {}}
    ok = True
    for k, q in enumerate(SUMMARY_KEYS):
        xa = np.array([r["summary"][k] for r in a_runs])
        xb = np.array([r["summary"][k] for r in b_runs])
        sa, sb = xa.std(ddof=1) / np.sqrt(len(xa)), xb.std(ddof=1) / np.sqrt(len(xb))
        se = float(np.hypot(sa, sb))
        z = float((xb.mean() - xa.mean()) / se) if se > 0 else 0.0
        ok = ok and abs(z) <= 3.0
        out["quantities"][q] = {a_name: float(xa.mean()), a_name + "_se": float(sa),
                                b_name: float(xb.mean()), b_name + "_se": float(sb), "z": z}

    def ks(ha, hb):
        na, nb = ha.sum(), hb.sum()
        d = float(np.max(np.abs(np.cumsum(ha) / na - np.cumsum(hb) / nb)))
        return d, float(special.kolmogorov(d * np.sqrt(na * nb / (na + nb)))), int(na), int(nb)

    ha = sum(r["hist"] for r in a_runs)
    hb = sum(r["hist"] for r in b_runs)
    d, p, na, nb = ks(ha, hb)
    half = lambda R: ks(sum(r["hist"] for r in R[: len(R) // 2]), sum(r["hist"] for r in R[len(R) // 2:]))[0]
    ref = max(half(a_runs), half(b_runs))
    p_perm = _ks_permutation_p([r["hist"] for r in a_runs], [r["hist"] for r in b_runs])
    out["logm_ks"] = {"D": d, "p_particles": p, "p_runs_permutation": p_perm, "D_half_vs_half": ref,
                      "samples": [na, nb], "bins_dex": (LOGM_EDGES[1] - LOGM_EDGES[0]) / LOGM_EDGES[2]}
    out["within_tolerance"] = bool(ok and p_perm > 0.01)
    return out


def large_disk_ensemble_combine(paths):
    """Combine the parts written by large_disk_ensemble_part: mixed against
    GPU FP64, or against the oracle, over their common horizon."""
    import numpy as np
    runs = {"fp64": [], "oracle": [], "mixed": []}
    years = None
    for path in paths:
        z = np.load(path)
        years = int(z["years"]) if years is None else years
        if int(z["years"]) != years:
            raise ValueError("parts of different horizons")
        for key in z.files:
            if key.endswith("_summary"):
                base = key[: -len("_summary")]
                side = base.split("_")[0]
                runs[side].append({"seed": int(base.split("_")[1]), "summary": z[key],
                                   "hist": z[base + "_hist"], "events": int(z[base + "_events"]),
                                   "wall": float(z[base + "_wall"])})
    for v in runs.values():
        v.sort(key=lambda r: r["seed"])
    runs = {k: v for k, v in runs.items() if v}
    ref = "fp64" if "fp64" in runs else "oracle"
    if ref not in runs or "mixed" not in runs:
        raise ValueError("the parts hold no mixed runs, or no FP64 or oracle runs to compare them with")
    out = compare_ensembles_hist(runs[ref], runs["mixed"], ref, "mixed")
    out.update({"horizon_yr": years,
                f"{ref}_seeds": [r["seed"] for r in runs[ref]],
                "mixed_seeds": [r["seed"] for r in runs["mixed"]],
                "s_per_run": {k: float(np.mean([r["wall"] for r in v])) for k, v in runs.items()},
                "events_per_run": {k: float(np.mean([r["events"] for r in v])) for k, v in runs.items()}})
    seeds_ref = [r["seed"] for r in runs[ref]]
    if seeds_ref == [r["seed"] for r in runs["mixed"]] and len(seeds_ref) > 1:
        # the same seeds on both sides: collisions per run compared run by run
        d = np.array([m["events"] / a["events"] - 1.0 for a, m in zip(runs[ref], runs["mixed"])])
        se = float(d.std(ddof=1) / np.sqrt(len(d)))
        out["paired_collisions"] = {"rel_diff_mean": float(d.mean()), "rel_diff_se": se,
                                    "z": float(d.mean() / se) if se > 0 else 0.0}
    return out


HOST_THREADS_MAX = 16   # the host-CPU share of one GPU on the measurement boxes


def host_threads():
    """Threads for the CPU oracle: the CPUs this process may run on, at most
    the host share of one GPU."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, HOST_THREADS_MAX))


def cpu_info():
    """Model, the logical CPUs this process may use, and how many distinct
    physical cores (and threads per core) they are, from /proc/cpuinfo."""
    allowed = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else set()
    cores, cpu, phys, core = {}, None, None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f.read().split("\n\n"):
                kv = dict(x.split(":", 1) for x in line.splitlines() if ":" in x)
                kv = {k.strip(): v.strip() for k, v in kv.items()}
                if "processor" not in kv:
                    continue
                cpu = int(kv["processor"])
                if allowed and cpu not in allowed:
                    continue
                key = (kv.get("physical id", "0"), kv.get("core id", str(cpu)))
                cores.setdefault(key, []).append(cpu)
    except OSError:
        pass
    logical = sum(len(v) for v in cores.values())
    return {"model": cpu_model(), "logical_cpus_allowed": logical or (os.cpu_count() or 1),
            "physical_cores_allowed": len(cores) or None,
            "threads_per_core": (max(len(v) for v in cores.values()) if cores else None)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(work, target_s=12.0, one_thread_s=3.0):
    """The FP64 oracle on a bounded sample of cells of the same workload,
    threads over cells on every host core; then the same on one thread over
    a smaller sample.  Collisions/s and algorithmic pair evaluations/s."""
    import numpy as np

    import oracle as O
    from paper_2507_21239_amd import workloads as W

    threads = host_threads()
    rng = np.random.default_rng(7)
    sizes = np.diff(work["cells"]["cell_start"])
    n_cells = len(sizes)
    perm = rng.permutation(n_cells)

    def run(nthreads, budget, k):
        used, evs, ncells, evals = 0.0, 0, 0, 0.0
        while used < budget and ncells < n_cells:
            cells = np.sort(perm[ncells:ncells + k])
            sub = W.subset_cells(work, cells)
            part = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in sub["particles"].items()}
            t0 = time.perf_counter()
            out = O.collide_all(sub["params"], sub["cells"], 0, part, 0.0, EVENTS_PER_CELL,
                                threads=nthreads)
            used += time.perf_counter() - t0
            ev = out["stats"]["events"]
            evs += int(ev.sum())
            n = sizes[cells].astype("float64")
            evals += float((n * (n + 1) / 2).sum() + (ev * n).sum())
            ncells += len(cells)
            k = min(2 * k, n_cells - ncells) if used < budget / 4 else k
        return used, evs, ncells, evals

    used, evs, ncells, evals = run(threads, target_s, max(threads, 8))
    u1, e1, c1, p1 = run(1, one_thread_s, 2)
    info = cpu_info()
    return dict(value=evs / used, unit="collisions/s", cores=threads, kind="oracle",
                host=dict(info, threads_used=threads),
                sample=f"{ncells} of {n_cells} cells of the same workload, {EVENTS_PER_CELL} events "
                       f"each ({evs} events), FP64, {used:.1f} s wall",
                pair_evals_per_s=evals / used,
                one_thread={"collisions_per_s": e1 / u1, "pair_evals_per_s": p1 / u1,
                            "sample": f"{c1} cells, {e1} events, {u1:.1f} s"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-error", action="store_true", help="skip the error report")
    ap.add_argument("--modes", default="all",
                    help="all | headline | none (only the full step, for profiling) | "
                         "next (cost of the sigma_d histogram, the gridded gas, the "
                         "fragmentation criteria and the snapshots) | configs (per-configuration "
                         "rates, GPU forms and oracle) | ensemble (the large disk's 16-seed "
                         "ensembles, mixed vs GPU FP64 and vs the oracle) | ensemble-part (a "
                         "part of the FP64 / mixed ensemble, saved for --combine) | steady (the "
                         "large disk's steady state alone, for profiling) | lone (one cell "
                         "alone, --lone and --events, --steps launches, for instruction counters)")
    ap.add_argument("--no-full-step", action="store_true", help="skip the full-path measurement")
    ap.add_argument("--years", type=int, default=1000,
                    help="horizon of --modes ensemble (the large disk's 16-seed ensembles)")
    ap.add_argument("--part", default="0,16",
                    help="--modes ensemble-part: first seed and count of this part")
    ap.add_argument("--out", default="gpurun_out/ensemble_part.npz",
                    help="--modes ensemble-part: where the part is saved")
    ap.add_argument("--sides", default="fp64,mixed",
                    help="--modes ensemble-part: which of fp64, oracle, mixed to run (oracle "
                         "alone needs no GPU)")
    ap.add_argument("--same-seeds", action="store_true",
                    help="--modes ensemble-part: the mixed runs take the other sides' seeds")
    ap.add_argument("--combine", nargs="*", default=None,
                    help="combine saved ensemble parts (host only) and print the comparison")
    ap.add_argument("--oracle-steps", type=int, default=3,
                    help="ensemble mode: steps of the large disk's oracle comparison")
    ap.add_argument("--schedule", default=None,
                    help="SMALL_MAX,GRID_PER_CU: fixed batched schedule instead of the autotuner "
                         "(profiling runs, so that no tuning trials enter the kernel statistics)")
    ap.add_argument("--lone", default="200",
                    help="--modes lone: the cell, N or N,n_comp")
    ap.add_argument("--events", type=int, default=EVENTS_PER_CELL,
                    help="--modes lone: events per collision launch")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the HBM counter calibration copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (cells would shard "
              "by contiguous ranges of radial zones)", file=sys.stderr)
        sys.exit(2)
    if args.combine:
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "large_disk_ensemble_combined": large_disk_ensemble_combine(args.combine)}),
              flush=True)
        return
    sides = tuple(x for x in args.sides.split(",") if x)
    if not sides or set(sides) - {"fp64", "oracle", "mixed"}:
        print("--sides takes fp64, oracle and mixed", file=sys.stderr)
        sys.exit(2)
    if args.modes == "ensemble-part" and sides == ("oracle",):
        first, count = (int(x) for x in args.part.split(","))
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "large_disk_ensemble_part": large_disk_ensemble_part(
                              first, count, args.years, args.out, sides=sides)}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2507_21239_amd import workloads as W

    assert torch.cuda.is_available(), "no GPU"
    global FIXED_SCHEDULE
    if args.schedule:
        sm, g = (int(x) for x in args.schedule.split(","))
        FIXED_SCHEDULE = (sm, g)
    if args.copy_calibration:
        copy_calibration()
        return
    work = W.c4_batched(seed=0, events=EVENTS_PER_CELL)
    counts = np.diff(work["cells"]["cell_start"])
    evals = pair_evals(counts, EVENTS_PER_CELL)
    log("workload", len(counts), "cells", int(counts.sum()), "particles", f"{evals:.3e} pair evals/step")

    if args.modes == "next":
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "next_rows": next_rows(args.steps, args.warmup)}), flush=True)
        return
    if args.modes == "configs":
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "cpu_model": cpu_model(), "configs": configs_table(args.steps)}),
              flush=True)
        return
    if args.modes == "ensemble":
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "large_disk_ensemble": large_disk_ensemble(
                              years=args.years, oracle_steps=args.oracle_steps)}), flush=True)
        return
    if args.modes == "ensemble-part":
        first, count = (int(x) for x in args.part.split(","))
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "large_disk_ensemble_part": large_disk_ensemble_part(
                              first, count, args.years, args.out, sides=sides,
                              same_seeds=args.same_seeds)}), flush=True)
        return
    if args.modes == "lone":
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "lone_cell": lone_counting(args.lone, args.events, args.steps)}),
              flush=True)
        return
    if args.modes == "steady":
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "steady_state": steady_state(args.steps)}), flush=True)
        return
    if args.modes == "none":
        fs = full_step(args.steps, args.warmup, steady=False)
        print(json.dumps({"metric": METRIC, "value": None, "unit": "collisions/s",
                          "full_step": fs}), flush=True)
        return
    modes = [("mixed", "batched")] if args.modes == "headline" else \
        [("fp64", "plain"), ("fp64", "batched"), ("mixed", "plain"), ("mixed", "batched")]
    res = {}
    for precision, schedule in modes:
        log("timing", precision, schedule)
        r = run_mode(work, precision, schedule, args.steps, args.warmup)
        r["collisions_per_s"] = r["events"] / r["wall_s"]
        r["pair_evals_per_s"] = evals * args.steps / r["wall_s"]
        res[f"{precision}_{schedule}"] = r
        log(precision, schedule, f"{r['ms_per_step']:.3f} ms/step", f"{r['collisions_per_s']:.3e} coll/s")
    head = res["mixed_batched"]
    achieved = F_PAIR * evals / (head["kernel_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": head["collisions_per_s"],
        "unit": "collisions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision": "FP32 pair rates; FP64 masses, prefix sums, row-sum state and time",
        "data": "synthetic",
        "config": {"workload": "batched collision step: 4096 cells, counts log-uniform [64,1024], "
                               "masses log-uniform 1e-12..1e2 g, random gas, 1000 events/cell",
                   "cells": int(len(counts)), "particles": int(counts.sum()),
                   "events_per_cell": EVENTS_PER_CELL, "schedule": "batched"},
        "pair_evals_per_s": head["pair_evals_per_s"],
        "forms": {k: {"collisions_per_s": v["collisions_per_s"], "pair_evals_per_s": v["pair_evals_per_s"],
                      "ms_per_step": v["ms_per_step"], "kernel_ms": v["kernel_ms"],
                      "tuned_schedule": v["schedule"]} for k, v in res.items()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic_bytes(),
                     "kernel": "collide_batched<float>", "flops_per_pair": F_PAIR,
                     "pair_evals_per_launch": evals,
                     "executed_pair_evals_per_launch": executed_pair_evals(counts, EVENTS_PER_CELL),
                     "valu_busy": issue_rate()[0],
                     "valu_insts_per_collision": issue_rate()[1]},
    }
    if "fp64_plain" in res:
        out["speedup_mixed_batched_vs_fp64_plain"] = head["collisions_per_s"] / res["fp64_plain"]["collisions_per_s"]
    if not args.no_full_step:
        log("full step on the large disk")
        out["full_step"] = full_step(args.steps, args.warmup)
        log("full step", f"{out['full_step']['ms_per_step']:.3f} ms/step",
            f"bin {out['full_step']['bin_ms']:.3f} ms",
            f"late {out['full_step']['late_window']['ms_per_step']:.3f} ms/step",
            f"steady {out['full_step']['steady_window']['ms_per_step']:.3f} ms/step")
        log("lone cells")
        out["lone_cell"] = lone_cells()
    if not args.no_error:
        log("error report")
        out["error"] = error_report(work)
        log("error report: ensembles of the 1e5 disk, oracle vs mixed")
        out["error"]["ensemble"] = ensemble_report()
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(work)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
