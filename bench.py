"""Benchmark of the hybrid-PIC step on one MI355X.

Headline: the largest single-GPU workload, a gold slab 250 um thick in a
512^3 grid of 0.5 um cells with 2e8 macro-electrons (T_hot = 10.8 MeV, 2 um
spot, 10 fs steps, paper reflux, 128x180 tally) in FP32-mixed precision,
and the same workload in FP64 on the same GPU (the metric compares the
two).  Also timed: the 256^3 slab with 1e8 electrons (FP32-mixed and FP64)
and the 256x128x128 slab with 2e7 electrons (FP64 and FP32-mixed), the
64-run serving scan (p50 / p99 latency) and the FP64 CPU oracle on a bounded
sample.  Inputs are synthetic (`workloads`).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only NAMES]
                    [--no-cpu] [--no-serve] [--opt-in] [--model] [--copy-probe]

Every workload first runs its injection window (1 ps) untimed, whatever W
is, and reports that window's rate separately (`injection_phase`); then W
warmup steps and K timed steps, inputs resident in HBM.  `value` is alive
electron-steps (the electrons alive at the start of each timed step, summed;
an exact device counter) over the wall time of the K steps.

`roofline` is the particle kernel's algorithmic bytes per launch (the
electron records read and the changed fields written) over its mean launch
duration, from HIP events recorded around every launch on the run's stream
during the timed steps.  `traffic` is the HBM bytes per launch that
rocprofv3's FETCH_SIZE and WRITE_SIZE counters gave for the same kernel on
the same workload and step window (the summary under profiles/), scaled by
the copy-kernel factors, or null when that summary was taken on other
kernel sources or another window.  `valu_roofline` sets the same kernel
against its VALU issue rate: wave-level VALU instructions per launch
(rocprofv3's SQ_INSTS_VALU, from a summary under profiles/ with the same
guards) over the live launch duration, against one 64-lane instruction
per SIMD every 4 cycles (the FP64 vector peak of 78.6 TFLOP/s over 128
flops per wave-level FMA: 6.14e11 per second).  `step_roofline` is the
whole step's algorithmic bytes (particles, sort, grid) over the step's
wall time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK = 78.6e12 / 128          # wave-level VALU instructions per second (1024 SIMDs, 4 cycles each)
METRIC = "macro-electron steps/s (FP32-mixed vs FP64, same GPU); p50/p99 scan-run latency"

# (name, workload function, precision, description)
WORKLOADS = (
    ("gold_512cube_2e8_fp32", "config_huge", 1, "gold slab 250 um, 512^3 cells of 0.5 um, 2e8 macro-electrons, "
                                  "T_hot 10.8 MeV (1e22 W/cm^2), 2 um spot, 30 deg cone, dt 10 fs, "
                                  "paper reflux, 128x180 tally"),
    ("gold_512cube_2e8_fp64", "config_huge", 0, None),
    ("gold_256cube_1e8_fp32", "config_mixed_large", 1, "gold slab x in [2, 254] um, 256^3 cells of 1 um, 1e8 "
                                         "macro-electrons, T_hot 10.8 MeV, 5 um spot, 30 deg cone, "
                                         "dt 20 fs, 1 % energy loss per reflux, 64x90 tally"),
    ("gold_256cube_1e8_fp64", "config_mixed_large", 0, None),
    ("gold_256x128x128_2e7_fp64", "config_fp64_large", 0, "gold slab 200 um, 256x128x128 cells of 1 um, 2e7 "
                                        "macro-electrons, T_hot 3.4 MeV (1e21 W/cm^2), 3 um spot, "
                                        "40 deg cone, dt 20 fs, paper reflux, 64x90 tally"),
    ("gold_256x128x128_2e7_fp32", "config_fp64_large", 1, None),
)

KERNEL_SOURCES = ("paper_2107_01723_amd/csrc/hyb_kernels.hip", "paper_2107_01723_amd/csrc/hyb_internal.h",
                  "paper_2107_01723_amd/csrc/hyb_solid.h")


def record_bytes(precision: int) -> tuple[int, int]:
    """Algorithmic bytes per electron-step of the particle kernel: the
    electron's record is read (cell and id u32, offsets (3), u (3), w / w_ref
    and tau in the run's precision) and its changed fields are written back
    (cell, offsets, u, tau; the id and weight do not change)."""
    t = 8 if precision == 0 else 4
    return 8 + 8 * t, 4 + 7 * t


def step_bytes(precision: int, electrons: float, nodes: int, solid_cells: int, n_sub: int) -> float:
    """Algorithmic bytes of one whole step: the particle kernel (above), the
    tile sort (every record read and written once), and the grid: the step's
    current and heat accumulators cleared (3 int64 per node, 1 per cell),
    Ohm's law per sub-cycle (B and j read, E written, eta once per cell),
    Faraday's law per sub-cycle (E and B read, B written) and the heating of
    the solid cells (j at the cell's edges, Te, Ti, eta and heat read; Te,
    Ti and eta written)."""
    t = 8 if precision == 0 else 4
    rd, wr = record_bytes(precision)
    rec = 8 + 8 * t
    per_node = 3 * 8 + n_sub * ((3 * t + 3 * 8 + 3 * t) + (3 * t + 3 * t + 3 * t))
    return electrons * (rd + wr + 2 * rec) + nodes * (per_node + 8) + solid_cells * (3 * 8 + 4 * 8 + 3 * 8)


def kernel_digest() -> str:
    """Digest of the device sources without their comments and blank lines
    (what the compiler sees); a counter summary holds the digest of the
    kernels it was taken on."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = [ln.split("//", 1)[0].rstrip() for ln in src.splitlines()]
        h.update("\n".join(ln for ln in code if ln.strip()).encode())
    return h.hexdigest()[:16]


def counted_traffic(name: str, window: tuple[int, int]):
    """HBM bytes per particle-kernel launch (FETCH_SIZE + WRITE_SIZE, scaled
    by the copy-probe factors) from the committed counter summary of this
    workload, or None when it is missing, was taken on other kernel sources
    or on another step window."""
    path = os.path.join(ROOT, "profiles", f"particle_kernel_hbm_bytes_{name}.txt")
    try:
        with open(path) as fh:
            kv = dict(ln.split(":", 1) for ln in fh if ":" in ln and not ln.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_digest") != kernel_digest() or kv.get("window") != f"{window[0]}-{window[1]}":
        return None
    v = kv.get("hbm_bytes_per_launch")
    return int(float(v)) if v else None


def counted_valu(name: str, window: tuple[int, int]):
    """Wave-level VALU instructions per particle-kernel launch (SQ_INSTS_VALU)
    from the committed counter summary of this workload, or None when it is
    missing, was taken on other kernel sources or on another step window."""
    path = os.path.join(ROOT, "profiles", f"particle_kernel_valu_{name}.txt")
    try:
        with open(path) as fh:
            kv = dict(ln.split(":", 1) for ln in fh if ":" in ln and not ln.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_digest") != kernel_digest() or kv.get("window") != f"{window[0]}-{window[1]}":
        return None
    v = kv.get("valu_insts_per_launch")
    return float(v) if v else None


def injection_steps(cfg, srcs) -> int:
    return max(int(math.floor(s["t_end"] / cfg["dt"] + 0.5)) for s in srcs)


def time_run(P, name, cfg, srcs, steps, warmup):
    """Injection window untimed (its rate reported apart), warmup, then the
    timed steps with HIP events around every particle-kernel launch."""
    import torch
    run = P.Run(cfg, device=0)
    for s in srcs:
        run.inject(s)
    info = run.info()
    n_inj = injection_steps(cfg, srcs)
    run.timing(True)
    torch.cuda.synchronize()
    start = time.perf_counter()
    run.step(n_inj)
    torch.cuda.synchronize()
    wall_inj = time.perf_counter() - start
    kms_inj, nl_inj = run.timing_get()
    t_inj = run.tally()
    run.step(warmup)
    run.timing_get()
    t0 = run.tally()
    torch.cuda.synchronize()
    start = time.perf_counter()
    run.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - start
    kms, nl = run.timing_get()
    t1 = run.tally()
    run.close()
    del run
    torch.cuda.empty_cache()
    es_inj = t_inj["counters"]["n_electron_steps"]
    es = t1["counters"]["n_electron_steps"] - t0["counters"]["n_electron_steps"]
    prec = cfg["precision"]
    kernel_ms = kms / max(nl, 1)
    per_launch = es / steps
    rd, wr = record_bytes(prec)
    achieved = (rd + wr) * per_launch / (kernel_ms * 1e-3) / 1e9
    window = (n_inj + warmup, n_inj + warmup + steps)
    traffic = counted_traffic(name, window)
    valu = counted_valu(name, window)
    valu_roof = None
    if valu:
        va = valu / (kernel_ms * 1e-3)
        valu_roof = dict(bound="alu", achieved=round(va, -6), peak=round(VALU_PEAK, -6), unit="wave-instr/s",
                         frac=round(va / VALU_PEAK, 4), insts_per_electron_step=round(64 * valu / per_launch, 1),
                         kernel="k_particle")
    solid = (round(cfg["x_hi"] / cfg["dx"]) - round(cfg["x_lo"] / cfg["dx"])) * cfg["ny"] * cfg["nz"]
    sb = step_bytes(prec, per_launch, info["nodes"], solid, info["n_sub"])
    led = t1["ledger"]
    out = (t1["kinetic"] + led["field_loss"] - led["field_gain"] + led["ionisation"] + led["stopped"]
           + led["rad_discrete"] + led["rad_subcut"] + led["escaped"] + led["reflux"] + led["residual"])
    return dict(
        value=round(es / wall, 1), ms_per_step=round(1e3 * wall / steps, 4), steps=steps, warmup=warmup,
        timed_steps=list(window), alive_mean=round(per_launch, 1),
        particle_kernel_ms=round(kernel_ms, 4), particle_kernel_launches=nl,
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                      bytes_per_electron_step=rd + wr, kernel="k_particle"),
        valu_roofline=valu_roof,
        step_roofline=dict(bytes_per_step=round(sb), achieved=round(sb / (wall / steps) / 1e9, 1),
                           peak=HBM_PEAK_GBS, unit="GB/s", frac=round(sb / (wall / steps) / 1e9 / HBM_PEAK_GBS, 4)),
        injection_phase=dict(steps=n_inj, ms_per_step=round(1e3 * wall_inj / n_inj, 4),
                             value=round(es_inj / wall_inj, 1),
                             particle_kernel_ms=round(kms_inj / max(nl_inj, 1), 4),
                             alive_end=t_inj["n_alive"]),
        n_sub=info["n_sub"], conversion=t1["conversion"], n_alive_end=t1["n_alive"],
        ledger_closure=abs(led["injected"] - out) / led["injected"],
        n_delta=t1["counters"]["n_delta"], n_delta_lost=t1["counters"]["n_delta_lost"])


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline():
    """The FP64 oracle, as it stands, on the host's cores (one process; its
    NumPy work is single-threaded): (1) the whole small workload (1e4
    electrons, 32x16x16 cells, 200 steps); (2) a sample of the headline
    workload: its material, cells, time step and source, 5e5 electrons
    injected in one step (untimed) on a 512x64x64 part of its grid around
    the spot, then timed steps, with the particle part and the grid update
    timed apart (electron-steps/s and cell-steps/s), and the whole 2e8 /
    512^3 step extrapolated from the two rates."""
    import copy
    import workloads as W
    from oracle import OracleRun

    def timed(ora, nsteps):
        acc = {"grid": 0.0}
        gu = ora.grid_update

        def wrapped():
            t = time.perf_counter()
            gu()
            acc["grid"] += time.perf_counter() - t
        ora.grid_update = wrapped
        es0 = ora.counters["n_electron_steps"]
        t = time.perf_counter()
        ora.run(nsteps)
        tot = time.perf_counter() - t
        return tot, acc["grid"], ora.counters["n_electron_steps"] - es0

    cfg, srcs, nsteps = W.config_small()
    ora = OracleRun(cfg)
    ora.add_source(srcs[0])
    tot1, grid1, es1 = timed(ora, nsteps)
    cells1 = cfg["nx"] * cfg["ny"] * cfg["nz"]

    cfg5, srcs5, _ = W.config_huge()
    c = copy.deepcopy(cfg5)
    c.update(ny=64, nz=64, max_particles=500_000)
    s = copy.deepcopy(srcs5[0])
    s.update(n_macro=500_000, t_end=c["dt"], y0=16e-6, z0=16e-6)
    ora = OracleRun(c)
    ora.add_source(s)
    ora.step()
    k = 8
    tot5, grid5, es5 = timed(ora, k)
    cells5 = c["nx"] * c["ny"] * c["nz"]
    p_rate = es5 / (tot5 - grid5)
    c_rate = cells5 * k / grid5
    full_cells = cfg5["nx"] * cfg5["ny"] * cfg5["nz"]
    extrap = 2e8 / p_rate + full_cells / c_rate
    return dict(
        value=round(p_rate, 1), unit="macro-electron steps/s", cores=1, kind="oracle",
        sample=(f"FP64 oracle on one core: the headline workload's physics, cells and source, 5e5 "
                f"electrons on a 512x64x64 part of its grid, {k} timed steps; value = particle "
                f"part only ({tot5 - grid5:.1f} s); grid update {c_rate:.3e} cell-steps/s "
                f"({grid5:.1f} s); the whole small workload (1e4 electrons, 32x16x16 cells, "
                f"{nsteps} steps) in {tot1:.1f} s"),
        cpu_model=_cpu_model(), os_cpu_count=os.cpu_count(),
        headline_sample=dict(electron_steps_per_s=round(p_rate, 1), cell_steps_per_s=round(c_rate, 1),
                             electron_steps=es5, cells=cells5, steps=k,
                             particle_s=round(tot5 - grid5, 2), grid_s=round(grid5, 2),
                             full_step_s_extrapolated=round(extrap, 1)),
        small_workload=dict(electron_steps_per_s=round(es1 / tot1, 1),
                            particle_electron_steps_per_s=round(es1 / (tot1 - grid1), 1),
                            cell_steps_per_s=round(cells1 * nsteps / grid1, 1), wall_s=round(tot1, 2),
                            electron_steps=es1, steps=nsteps))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--only", default="", help="comma-separated workload names (default: all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--model", action="store_true",
                    help="also time the energy-partition model over the intensity-Z plane")
    ap.add_argument("--opt-in", action="store_true",
                    help="also time the 2e7-electron FP64 workload with delta rays, with eq. F_sigma "
                         "and with the Urban-type scatter")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 512 MiB with torch (reference kernel for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported (the step runs "
              f"on a single GPU)", file=sys.stderr)
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

    only = [x for x in a.only.split(",") if x]
    unknown = [x for x in only if x not in [w[0] for w in WORKLOADS]]
    if unknown:
        print(f"bench.py: unknown workload(s) {unknown}; known: {[w[0] for w in WORKLOADS]}", file=sys.stderr)
        sys.exit(2)
    res, desc = {}, {}
    for name, fn, prec, d in WORKLOADS:
        if d:
            desc[name.rsplit("_", 1)[0]] = d
        if only and name not in only:
            continue
        cfg, srcs, _ = getattr(W, fn)()
        cfg = dict(cfg, precision=prec)
        print(f"# {name}: {cfg['nx']}x{cfg['ny']}x{cfg['nz']}, {srcs[0]['n_macro']} electrons, "
              f"injection window + {a.warmup} warmup + {a.steps} timed steps", file=sys.stderr, flush=True)
        r = time_run(P, name, cfg, srcs, a.steps, a.warmup)
        res[name] = r
        print(f"# {name}: {r['ms_per_step']:.3f} ms/step, {r['value']:.3e} electron-steps/s, particle kernel "
              f"{r['particle_kernel_ms']:.3f} ms ({r['roofline']['frac']:.3f} of HBM); injection window "
              f"{r['injection_phase']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    opt_in = {}
    if a.opt_in:
        for nm, bit, extra in (("delta_rays", W.PHYS_DELTA, 1.5), ("f_sigma", W.PHYS_FSIGMA, 1.0),
                               ("urban_scatter", W.PHYS_URBAN, 1.0)):
            cfg, srcs, _ = W.config_fp64_large()
            cfg = dict(cfg, physics=cfg["physics"] | bit, max_particles=int(cfg["max_particles"] * extra))
            r = time_run(P, "gold_256x128x128_2e7_fp64_" + nm, cfg, srcs, a.steps, a.warmup)
            opt_in[nm] = {k: r[k] for k in ("value", "ms_per_step", "particle_kernel_ms", "alive_mean",
                                            "roofline", "ledger_closure", "n_delta", "n_delta_lost")}
            print(f"# gold_256x128x128_2e7_fp64 + {nm}: {r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
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
    serving = None
    if not a.no_serve:
        from paper_2107_01723_amd import serve
        print("# serving: 64-run scan (Poisson arrivals, 2 runs/s)", file=sys.stderr, flush=True)
        sv = serve.run_scan(W.scan_runs(64, seed=0), verbose=True)
        serving = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sv.items() if k != "results"}
        print(f"# serving: p50 {sv['p50_s']:.2f} s, p99 {sv['p99_s']:.2f} s, "
              f"{sv['electron_steps_per_s']:.3e} electron-steps/s", file=sys.stderr, flush=True)
    cpu = None
    if not a.no_cpu:
        print("# cpu oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
        print(f"# cpu oracle: {cpu['value']:.3e} electron-steps/s (particles), "
              f"{cpu['headline_sample']['cell_steps_per_s']:.3e} cell-steps/s", file=sys.stderr, flush=True)

    head = res.get("gold_512cube_2e8_fp32") or next(iter(res.values()), None)
    hname = "gold_512cube_2e8_fp32" if "gold_512cube_2e8_fp32" in res else (next(iter(res)) if res else None)
    line = {"metric": METRIC, "unit": "macro-electron steps/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic"}
    if head:
        fp32 = hname.endswith("fp32")
        line.update(
            value=head["value"], ms_per_step=head["ms_per_step"],
            dtype="f32" if fp32 else "f64",
            config={"workload": f"{hname}: {desc[hname.rsplit('_', 1)[0]]}; "
                                + ("FP32-mixed (FP32 particle state, push and table sampling; FP64 heating "
                                   "and resistivity; int64 fixed-point current, ledger and tallies)" if fp32
                                   else "FP64 throughout (int64 fixed-point current, ledger and tallies)")
                                + f"; timed after the untimed {head['injection_phase']['steps']}-step "
                                  f"injection window",
                    "timed_steps": head["timed_steps"], "alive_mean": head["alive_mean"]},
            roofline=head["roofline"], valu_roofline=head["valu_roofline"], step_roofline=head["step_roofline"],
            particle_kernel_ms=head["particle_kernel_ms"], injection_phase=head["injection_phase"],
            ledger_closure=head["ledger_closure"])
        if hname == "gold_512cube_2e8_fp32" and "gold_512cube_2e8_fp64" in res:
            f64 = res["gold_512cube_2e8_fp64"]
            line["fp64"] = {k: f64[k] for k in ("value", "ms_per_step", "particle_kernel_ms", "roofline",
                                                "valu_roofline", "step_roofline", "injection_phase",
                                                "ledger_closure")}
            line["mixed_over_fp64"] = round(head["value"] / f64["value"], 3)
        line["workloads"] = {k: v for k, v in res.items() if k not in (hname, "gold_512cube_2e8_fp64" if hname == "gold_512cube_2e8_fp32" else "")}
        ratios = {}
        for c in {k.rsplit("_", 1)[0] for k in res}:
            if f"{c}_fp32" in res and f"{c}_fp64" in res:
                ratios[c] = round(res[f"{c}_fp32"]["value"] / res[f"{c}_fp64"]["value"], 3)
        line["mixed_over_fp64_by_workload"] = ratios
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
