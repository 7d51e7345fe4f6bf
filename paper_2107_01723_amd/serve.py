"""Continuous-batching driver for parameter-scan runs on one GPU.

Requests (independent hybrid-PIC runs) arrive over wall-clock time.  Arrived
requests wait in a FIFO queue and are admitted to the engine as soon as a
slot and enough device memory are free; every engine tick advances all
resident runs by one step with batched kernels (one launch per phase for all
of them, replayed as a HIP graph), so runs admitted while others are running
overlap on the device.  Finished runs are tallied and retired, which frees
their slot and memory for the queue.  Latency is arrival -> tally returned.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from .hyb import Engine


def run_scan(requests, ticks_per_poll: int = 8, max_runs: int = 64, hbm_budget: int = 0,
             time_scale: float = 1.0, verbose: bool = False, device: int = 0) -> dict:
    """requests: dicts with keys arrival [s], cfg, srcs, steps (see
    workloads.scan_runs).  Returns latency percentiles and throughput."""
    import torch

    eng = Engine(device=device, hbm_budget=hbm_budget, max_runs=max_runs)
    order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival"])
    pending = list(order)          # not yet arrived
    queue = []                     # arrived, waiting for admission
    resident = {}                  # run handle value -> (request index, Run)
    lat, done_at, results = {}, {}, {}
    particle_steps = 0            # electrons alive at the start of each step, summed
    t0 = time.perf_counter()
    max_res = 0
    while pending or queue or resident:
        now = (time.perf_counter() - t0) / time_scale
        while pending and requests[pending[0]]["arrival"] <= now:
            queue.append(pending.pop(0))
        while queue:
            i = queue[0]
            rq = requests[i]
            r = eng.admit(rq["cfg"], rq["srcs"], rq["steps"])
            if r is None:
                break
            queue.pop(0)
            resident[r.h.value] = (i, r)
        max_res = max(max_res, len(resident))
        if resident:
            eng.step(ticks_per_poll)
            for r in eng.poll():
                i, _ = resident.pop(r.h.value)
                t = r.tally()
                now = (time.perf_counter() - t0) / time_scale
                lat[i] = now - requests[i]["arrival"]
                results[i] = dict(conversion=t["conversion"], n_alive=t["n_alive"], step=t["step"],
                                  ledger=t["ledger"])
                particle_steps += t["counters"]["n_electron_steps"]
                eng.retire(r)
                if verbose:
                    print(f"# run {i:3d} done: latency {lat[i]:7.2f} s, resident {len(resident)}, "
                          f"queued {len(queue)}", file=sys.stderr, flush=True)
        elif pending:
            time.sleep(max(0.0, min(0.05, requests[pending[0]]["arrival"] - now)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    eng.close()
    L = np.array([lat[i] for i in sorted(lat)])
    return dict(runs=len(L), p50_s=float(np.percentile(L, 50)), p99_s=float(np.percentile(L, 99)),
                max_s=float(L.max()), wall_s=wall, max_resident=max_res,
                electron_steps=particle_steps, electron_steps_per_s=particle_steps / wall, results=results)
