"""Helpers of the GPU parity tests: build matched oracle/GPU runs and compare
their states particle by particle."""
import numpy as np

import workloads as W
from oracle import OracleRun


def oracle_at(cfg, srcs, nsteps):
    r = OracleRun(cfg)
    for s in srcs:
        r.add_source(s)
    r.run(nsteps)
    return r


def gpu_from_oracle(P, cfg, srcs, ora, device=0):
    run = P.Run(cfg, device=device)
    for s in srcs:
        run.inject(s)
    run.set_state(ora.state())
    return run


def match(got, ref):
    """Index arrays that align the two states by particle id."""
    gi = np.argsort(got["ids"], kind="stable")
    ri = np.argsort(ref["ids"], kind="stable")
    return gi, ri


def particle_errors(got, ref, dx):
    """Per-particle errors of particles alive in both: |dx|/dx (position),
    |dp|/|p| (momentum) and |dtau|/max(1, tau).  Returns (errs dict, ids
    alive in only one of the two)."""
    gids, rids = set(got["ids"].tolist()), set(ref["ids"].tolist())
    both = np.array(sorted(gids & rids), dtype=np.int64)
    only = sorted(gids ^ rids)
    gsel = np.isin(got["ids"], both)
    rsel = np.isin(ref["ids"], both)
    gi = np.argsort(got["ids"][gsel])
    ri = np.argsort(ref["ids"][rsel])
    gp, rp = got["p"][gsel][gi], ref["p"][rsel][ri]
    gx, rx = got["pos"][gsel][gi], ref["pos"][rsel][ri]
    gt, rt = got["tau"][gsel][gi], ref["tau"][rsel][ri]
    e = dict(
        ids=both,
        pos=np.max(np.abs(gx - rx), axis=1) / dx if len(both) else np.zeros(0),
        p=np.linalg.norm(gp - rp, axis=1) / np.maximum(np.linalg.norm(rp, axis=1), 1e-300),
        tau=np.abs(gt - rt) / np.maximum(1.0, np.abs(rt)),
        w=np.abs(got["w"][gsel][gi] - ref["w"][rsel][ri]) / ref["w"][rsel][ri],
    )
    if "tau_d" in got and "tau_d" in ref:
        gd, rd = got["tau_d"][gsel][gi], ref["tau_d"][rsel][ri]
        e["tau_d"] = np.abs(gd - rd) / np.maximum(1.0, np.abs(rd))
    return e, only


def field_rel(a, b):
    """max |a - b| / max |b| over the three components."""
    num = max(np.max(np.abs(x - y)) for x, y in zip(a, b))
    den = max(np.max(np.abs(y)) for y in b)
    return num / den if den > 0 else num


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


def ledger_delta(before, after):
    return {k: after[k] - before[k] for k in after}


def small_config(n_macro=10000, precision=W.FP64, **over):
    cfg, srcs, steps = W.config_small()
    cfg["precision"] = precision
    srcs[0]["n_macro"] = n_macro
    cfg["max_particles"] = max(1024, n_macro)
    cfg.update(over)
    return cfg, srcs, steps
