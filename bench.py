"""Benchmark of the hybrid-PIC step on one MI355X.

Workload: the FP64 gold-slab run of 2e7 macro-electrons on a 256x128x128
grid of 1 um cells (T_hot = 3.4 MeV, 3 um spot, 40 deg cone, 20 fs steps,
paper reflux, 64x90 tally), synthetic inputs from `workloads`.  Warmup steps
cover the 1 ps injection, so the timed steps carry the full particle load.
The same workload is also timed in FP32-mixed precision.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--serve] [--opt-in]

Prints one JSON line.  `value` is FP64 macro-electron steps per second
(alive electrons x steps / wall time of the timed steps, inputs resident in
HBM).  `roofline` is the particle kernel's algorithmic bytes per launch over
its mean duration, measured with HIP events on the run's stream; its
`traffic` is the HBM bytes per launch that rocprofv3's FETCH_SIZE and
WRITE_SIZE counters gave for the same kernel (per electron, from the summary
under profiles/, times this run's mean alive count), or null when that
summary was taken on other kernel sources.

`--opt-in` also times the same FP64 workload with each opt-in process of
the paper switched on (delta rays with the restricted loss; the eq. F_sigma
enhancement; the Urban-type elastic scatter in place of Davies) and reports
them under `opt_in`; the headline numbers are those of the default physics.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MEC2 = 8.1871057769e-14


def particle_bytes(precision: int) -> int:
    """Algorithmic bytes per particle-step of the particle kernel: the state
    is read once and written once (SoA: packed cell u32, 3 offsets, 3
    momenta, weight, optical depth, id u32; weight and id are not written)."""
    t = 8 if precision == 0 else 4
    read = 4 + 3 * t + 3 * t + t + t + 4
    write = 4 + 3 * t + 3 * t + t
    return read + write


KERNEL_SOURCES = ("paper_2107_01723_amd/csrc/hyb_kernels.hip", "paper_2107_01723_amd/csrc/hyb_internal.h",
                  "paper_2107_01723_amd/csrc/hyb_solid.h")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "particle_kernel_hbm_bytes_gold_slab_256x128x128_2e7.txt")


def kernel_digest() -> str:
    """Digest of the device sources; a counter summary holds the digest of
    the kernels it was taken on."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_bytes_per_electron(label: str):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by the copy-probe factors)
    per electron-step of the particle kernel, from the committed counter
    summary; None when the summary is missing or was taken on other kernels."""
    try:
        with open(COUNTER_SUMMARY) as fh:
            kv = dict(ln.split(":", 1) for ln in fh if ":" in ln and not ln.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_digest") != kernel_digest():
        return None
    v = kv.get(f"{label}_hbm_bytes_per_electron")
    return float(v) if v else None


def time_run(P, cfg, srcs, steps, warmup, label):
    import torch
    run = P.Run(cfg, device=0)
    for s in srcs:
        run.inject(s)
    run.step(warmup)
    t0 = run.tally()
    run.timing(True)
    torch.cuda.synchronize()
    start = time.perf_counter()
    run.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - start
    kms, nlaunch = run.timing_get()
    t1 = run.tally()
    alive = 0.5 * (t0["n_alive"] + t1["n_alive"])
    res = dict(label=label, wall_s=wall, ms_per_step=1e3 * wall / steps,
               particle_steps_per_s=alive * steps / wall, alive_mean=alive,
               kernel_ms=kms / max(nlaunch, 1), kernel_launches=nlaunch,
               conversion=t1["conversion"], n_alive_end=t1["n_alive"],
               n_delta=t1["counters"]["n_delta"] - t0["counters"]["n_delta"],
               n_delta_lost=t1["counters"]["n_delta_lost"])
    pb = particle_bytes(cfg["precision"])
    achieved = pb * alive / (res["kernel_ms"] * 1e-3) / 1e9
    bpe = counted_bytes_per_electron(label)
    traffic = None if bpe is None else round(bpe * alive)
    res["roofline"] = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                           bytes_per_particle_step=pb)
    led = t1["ledger"]
    out = (t1["kinetic"] + led["field_loss"] - led["field_gain"] + led["ionisation"] + led["stopped"]
           + led["rad_discrete"] + led["rad_subcut"] + led["escaped"] + led["reflux"] + led["residual"])
    res["ledger_closure"] = abs(led["injected"] - out) / led["injected"]
    run.close()
    return res


def cpu_baseline(cfg, srcs, n_macro=100_000, steps=12):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    full grid, n_macro electrons all injected in the first step (untimed),
    then `steps` timed steps on one core."""
    import copy
    from oracle import OracleRun
    c = copy.deepcopy(cfg)
    s = copy.deepcopy(srcs[0])
    s.update(n_macro=n_macro, t_start=0.0, t_end=c["dt"])
    ora = OracleRun(c)
    ora.add_source(s)
    ora.step()
    alive0 = int(ora.alive.sum())
    t0 = time.perf_counter()
    ora.run(steps)
    dt = time.perf_counter() - t0
    alive1 = int(ora.alive.sum())
    v = 0.5 * (alive0 + alive1) * steps / dt
    return dict(value=round(v, 1), unit="macro-electron steps/s", cores=1, kind="oracle",
                sample=f"FP64 oracle, full {c['nx']}x{c['ny']}x{c['nz']} grid, {n_macro} electrons "
                       f"injected in one step, {steps} timed steps ({dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--serve", action="store_true", help="also run the 64-run serving scan")
    ap.add_argument("--particles", type=int, default=0, help="override the macro-electron count")
    ap.add_argument("--model", action="store_true",
                    help="also time the energy-partition model over the intensity-Z plane")
    ap.add_argument("--opt-in", action="store_true",
                    help="also time the workload with delta rays, with eq. F_sigma and with the "
                         "Urban-type scatter (FP64)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 512 MiB with torch (reference kernel for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import workloads as W
    import paper_2107_01723_amd as P

    if a.copy_probe:
        # reference kernel for the HBM byte counters: one 512 MiB device copy
        # whose source was pushed out of the caches by writing 2 GiB elsewhere
        import torch
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        evict = torch.ones(512 << 20, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# copy probe: 512 MiB read + 512 MiB written", file=sys.stderr, flush=True)
        del src, dst, evict

    cfg, srcs, total_steps = W.config_fp64_large()
    if a.particles:
        cfg, srcs = W.scale_particles(cfg, srcs, a.particles)
    print(f"# workload FP64 {cfg['nx']}x{cfg['ny']}x{cfg['nz']}, {srcs[0]['n_macro']} electrons, "
          f"warmup {a.warmup} + {a.steps} timed steps", file=sys.stderr, flush=True)
    r64 = time_run(P, cfg, srcs, a.steps, a.warmup, "fp64")
    print(f"# fp64: {r64['ms_per_step']:.3f} ms/step, particle kernel {r64['kernel_ms']:.3f} ms, "
          f"{r64['particle_steps_per_s']:.3e} steps/s", file=sys.stderr, flush=True)
    r32 = None
    if not a.no_fp32:
        c32 = dict(cfg, precision=W.FP32_MIXED)
        r32 = time_run(P, c32, srcs, a.steps, a.warmup, "fp32_mixed")
        print(f"# fp32-mixed: {r32['ms_per_step']:.3f} ms/step, particle kernel {r32['kernel_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    opt_in = {}
    if a.opt_in:
        for name, bit, extra in (("delta_rays", W.PHYS_DELTA, 1.5), ("f_sigma", W.PHYS_FSIGMA, 1.0),
                                 ("urban_scatter", W.PHYS_URBAN, 1.0)):
            c = dict(cfg, physics=cfg["physics"] | bit, max_particles=int(cfg["max_particles"] * extra))
            r = time_run(P, c, srcs, a.steps, a.warmup, "fp64_" + name)
            opt_in[name] = {"value": round(r["particle_steps_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                            "particle_kernel_ms": round(r["kernel_ms"], 4), "alive_mean": r["alive_mean"],
                            "roofline": r["roofline"], "ledger_closure": r["ledger_closure"]}
            if bit == W.PHYS_DELTA:
                opt_in[name].update(delta_rays_timed=r["n_delta"], delta_rays_lost=r["n_delta_lost"])
            print(f"# fp64 + {name}: {r['ms_per_step']:.3f} ms/step, particle kernel {r['kernel_ms']:.3f} ms",
                  file=sys.stderr, flush=True)
    model = None
    if a.model:
        import numpy as np
        import torch
        m = W.model_inputs()
        I, Z = W.model_scan_grid()
        P.model_scan(m, I[:64], Z[:64])          # warm-up (module load)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = P.model_scan(m, I, Z)
        wall = time.perf_counter() - t0
        model = {"points": len(I), "rk4_steps_per_electron": m["nsteps"], "wall_ms": round(1e3 * wall, 3),
                 "electron_steps_per_s": round(3 * len(I) * m["nsteps"] / wall, 1),
                 "eta_e_gamma_range": [float(np.min(f[1])), float(np.max(f[1]))]}
        print(f"# model: {len(I)} points in {1e3 * wall:.2f} ms", file=sys.stderr, flush=True)
    serving = None
    if a.serve:
        from paper_2107_01723_amd import serve
        serving = serve.run_scan(W.scan_runs(64, seed=0), verbose=True)
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(cfg, srcs)
        print(f"# cpu oracle: {cpu['value']:.3e} steps/s", file=sys.stderr, flush=True)

    line = {
        "metric": "macro-electron steps/s (FP32-mixed vs FP64, same GPU); p50/p99 scan-run latency",
        "value": round(r64["particle_steps_per_s"], 1),
        "unit": "macro-electron steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gold slab 200 um, 256x128x128 cells of 1 um, 2e7 macro-electrons, "
                               "T_hot 3.4 MeV (1e21 W/cm^2), 3 um spot, 40 deg cone, dt 20 fs, "
                               "paper reflux, 64x90 tally, FP64",
                   "macro_electrons": srcs[0]["n_macro"], "alive_mean": r64["alive_mean"],
                   "grid": [cfg["nx"], cfg["ny"], cfg["nz"]]},
        "roofline": r64["roofline"],
        "particle_kernel_ms": round(r64["kernel_ms"], 4),
        "ledger_closure": r64["ledger_closure"],
    }
    if r32:
        line["fp32_mixed"] = {"value": round(r32["particle_steps_per_s"], 1),
                              "ms_per_step": round(r32["ms_per_step"], 4),
                              "particle_kernel_ms": round(r32["kernel_ms"], 4),
                              "roofline": r32["roofline"], "ledger_closure": r32["ledger_closure"]}
        line["mixed_over_fp64"] = round(r32["particle_steps_per_s"] / r64["particle_steps_per_s"], 3)
    if opt_in:
        line["opt_in"] = opt_in
    if model:
        line["model"] = model
    if serving:
        line["serving"] = serving
    if cpu:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
