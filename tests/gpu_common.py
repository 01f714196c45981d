"""Helpers shared by the GPU tests: run one workload through the HIP library
and through the CPU oracle on identical seeded inputs."""
from __future__ import annotations

import copy
import sys

import numpy as np

import oracle as O
from paper_2507_21239_amd import workloads as W


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def host_copy(part: dict) -> dict:
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in part.items()}


def run_oracle_explicit(work: dict, log_per_cell: int = 0, step: int = 0, threads: int = 0):
    part = host_copy(work["particles"])
    out = O.collide_all(work["params"], work["cells"], step, part, work["dt"], work["max_events"],
                        log_per_cell=log_per_cell, threads=threads)
    return part, out


def run_gpu_explicit(work: dict, precision: str, schedule: str, log_per_cell: int = 0,
                     n_steps: int = 1, batched_schedule=None):
    import torch
    from paper_2507_21239_amd import api
    say(work["name"], precision, schedule, "cells", len(work["cells"]["cell_start"]) - 1,
        "N", len(work["particles"]["m"]))
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision=precision, schedule=schedule)
    sim.bin(api.cells_to_device(work["cells"]))
    if batched_schedule is not None:
        sim.set_schedule(*batched_schedule)
    nc = len(work["cells"]["cell_start"]) - 1
    log = None
    if log_per_cell:
        log = torch.full((nc * log_per_cell * 4,), -7, dtype=torch.int32, device="cuda")
        sim.set_event_log(log, log_per_cell)
    sim.step(work["dt"], work["max_events"], n_steps)
    stats = sim.stats()
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in dev.items()}
    logh = log.cpu().numpy().reshape(nc, log_per_cell, 4) if log is not None else None
    sim.close()
    return host, stats, logh


def compare_logs(olog, ostats, glog):
    """Event sequences must agree exactly; entries past the last event of a
    cell must be untouched on the GPU."""
    nc, per = glog.shape[:2]
    bad = []
    for c in range(nc):
        ne = min(int(ostats["events"][c]), per)
        o = np.stack([olog[c]["i"][:ne], olog[c]["j"][:ne], olog[c]["outcome"][:ne]], axis=1)
        g = glog[c, :ne, :3]
        if not np.array_equal(o, g):
            k = int(np.argmax(np.any(o != g, axis=1)))
            bad.append((c, k, o[k].tolist(), g[k].tolist()))
        if ne < per and not np.all(glog[c, ne:, :] == -7):
            bad.append((c, "extra events on the GPU"))
    return bad


def edge_size_work(events: int = 200, seed: int = 3, precision_seed: int = 0) -> dict:
    """Explicit cells whose sizes hit every boundary of the kernel's layout:
    empty, one particle, wave multiples +-1, the one-wave / team switch
    (256 / 257), and the largest plain-schedule cell (1024)."""
    counts = [1, 0, 2, 3, 63, 64, 65, 127, 200, 255, 256, 257, 300, 511, 512, 513, 700, 1023, 1024]
    w = W.c4_batched(seed=seed, counts=counts, events=events, philox_seed=precision_seed)
    w["name"] = "edge_sizes"
    return w


def deepcopy(work: dict) -> dict:
    return copy.deepcopy(work)
