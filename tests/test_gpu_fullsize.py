"""GPU parity at the benchmark's full size, in the launch configuration
bench.py times: the gold slab of 256x128x128 cells with 2e7 macro-electrons
(FP64, and the same workload in FP32-mixed), and the 256^3 FP32-mixed slab
with 1e8 macro-electrons.

At this size the oracle cannot step the whole run, but every electron's step
depends only on its own state and the fields at the start of the step.  So a
sample of electrons is taken from the GPU state, stepped once by the oracle
in those fields, and compared with the same electrons after the GPU's step of
the whole population.  Quantities that involve all electrons are checked
through properties that hold at any size: the energy ledger closes, the
photon tallies add up to the radiated energy, and the particle buffer is in
tile order after each sort.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleRun

from parity_util import field_rel, particle_errors, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_01723_amd as P
    P.check_abi()
    return P


def _closure(t):
    led = t["ledger"]
    out = (t["kinetic"] + led["field_loss"] - led["field_gain"] + led["ionisation"] + led["stopped"]
           + led["rad_discrete"] + led["rad_subcut"] + led["escaped"] + led["reflux"] + led["residual"])
    return abs(led["injected"] - out) / led["injected"]


def _subset(st, ids):
    sel = np.isin(st["ids"], ids)
    return {k: (st[k][sel] if k in ("pos", "p", "w", "tau", "tau_d", "ids") else st[k]) for k in st}


@pytest.mark.parametrize("precision,n_pre,tol", [(W.FP64, 30, 1e-10), (W.FP64, 60, 1e-10),
                                                  (W.FP32_MIXED, 60, 1e-5)])
def test_fullsize_sampled_electrons(P, precision, n_pre, tol):
    """2000 electrons drawn from the full 2e7 population (during and after the
    injection), one step: oracle vs GPU per electron within the precision's
    bar; FP32 electrons whose discrete path differs are counted (<= 0.5 %)."""
    cfg, srcs, _ = W.config_fp64_large()
    cfg["precision"] = precision
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(n_pre)
    st0 = run.get_state()
    run.step(1)
    st1 = run.get_state()
    run.close()
    n0 = len(st0["ids"])
    print(f"  precision {precision}, step {n_pre}: {n0} electrons alive", flush=True)
    assert n0 > 5_000_000
    pick = np.random.default_rng(7).choice(n0, 2000, replace=False)
    ids = st0["ids"][pick]
    ora = OracleRun(cfg)
    ora.set_state(dict(_subset(st0, ids), step=st0["step"], next_id=st0["next_id"]))
    ora.step()
    ref = ora.state()
    got = _subset(st1, ids)
    err, only = particle_errors(got, ref, cfg["dx"])
    bad = (err["p"] > tol) | (err["pos"] > tol) | (err["tau"] > tol)
    nflip = int(np.sum(bad)) + len(only)
    print(f"  compared {len(err['ids'])}: max|dp|={err['p'][~bad].max():.2e} "
          f"max|dx|/dx={err['pos'][~bad].max():.2e} max|dtau|={err['tau'][~bad].max():.2e} "
          f"flips={nflip}", flush=True)
    assert len(err["ids"]) > 1800
    assert nflip <= (0 if precision == W.FP64 else 0.005 * len(ids)), (nflip, only[:10])
    assert err["w"].max() <= tol


@pytest.mark.parametrize("which,n_pre", [("c3", 25), ("c5", 40)])
def test_fullsize_sampled_electrons_fp32_large(P, which, n_pre):
    """FP32-mixed at the two large workloads, during the injection (the
    injection plane's tiles hold 1e5-1e6 electrons, so the workgroups carry
    LDS regions over many chunks and the chunks of the unsorted injected
    tail use every region): 2000 electrons drawn from the whole population,
    one step, oracle vs GPU within 1e-5 per electron, electrons whose
    discrete path differs counted (<= 0.5 %).  The oracle steps only the
    sample (no injection) and skips its grid update, which this step's
    particles do not see."""
    if which == "c3":
        cfg, srcs, _ = W.config_mixed_large()
    else:
        cfg, srcs, _ = W.config_huge()
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(n_pre)
    cap = run.tally()["n_alive"] + 1
    st0 = run.get_state(capacity=cap + srcs[0]["n_macro"] // 50)
    run.step(1)
    st1 = run.get_state(capacity=cap + 2 * srcs[0]["n_macro"] // 50)
    run.close()
    n0 = len(st0["ids"])
    print(f"  {which} step {n_pre}: {n0} electrons alive", flush=True)
    assert n0 > 20_000_000
    pick = np.random.default_rng(13).choice(n0, 2000, replace=False)
    ids = st0["ids"][pick]
    ora = OracleRun(cfg)
    ora.grid_update = lambda: None
    ora.set_state(dict(_subset(st0, ids), step=st0["step"], next_id=st0["next_id"]))
    del st0
    ora.step()
    ref = ora.state()
    got = _subset(st1, ids)
    del st1
    err, only = particle_errors(got, ref, cfg["dx"])
    tol = 1e-5
    bad = (err["p"] > tol) | (err["pos"] > tol) | (err["tau"] > tol)
    nflip = int(np.sum(bad)) + len(only)
    print(f"  compared {len(err['ids'])}: max|dp|={err['p'][~bad].max():.2e} "
          f"max|dx|/dx={err['pos'][~bad].max():.2e} max|dtau|={err['tau'][~bad].max():.2e} "
          f"flips={nflip}", flush=True)
    assert len(err["ids"]) > 1800
    assert nflip <= 0.005 * len(ids), (nflip, only[:10])
    assert err["w"].max() <= tol


def _check_run_properties(t, st):
    """Properties of a whole run at any size."""
    assert _closure(t) < 1e-6
    led = t["ledger"]
    # every photon's energy went to exactly one bin or flow slot
    radiated = float(np.sum(t["hist_E"])) + t["flow"][0] + t["flow"][2]
    assert radiated == pytest.approx(led["rad_discrete"], rel=1e-9)
    assert 0 <= led["photon_thr"] <= led["rad_discrete"] * (1 + 1e-12)
    assert t["counters"]["n_emitted"] > 0 and t["counters"]["n_reflux"] > 0


def test_fullsize_fp64_run_properties(P):
    """60 steps of the 2e7-electron FP64 workload (all of the 1 ps injection):
    ledger closure, tally sums and the tile order of the sorted buffer."""
    cfg, srcs, _ = W.config_fp64_large()
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(60)
    t = run.tally()
    st = run.get_state()
    run.close()
    print(f"  closure {_closure(t):.2e}, alive {t['n_alive']}", flush=True)
    _check_run_properties(t, st)
    assert len(st["ids"]) == t["n_alive"]
    # the buffer is in tile order after the step's sort (4^3-cell tiles, x fastest)
    c = np.floor(st["pos"] / cfg["dx"]).astype(np.int64)
    ntx, nty = cfg["nx"] // 4, cfg["ny"] // 4
    tile = (c[:, 0] >> 2) + ntx * ((c[:, 1] >> 2) + nty * (c[:, 2] >> 2))
    assert np.all(np.diff(tile) >= 0)
    # ids are unique
    assert len(np.unique(st["ids"])) == len(st["ids"])


def test_fullsize_fp32_256cube_properties(P):
    """The 1e8-electron FP32-mixed 256^3 workload through its injection:
    ledger closure and tally sums at full size."""
    cfg, srcs, _ = W.config_mixed_large()
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(55)
    t = run.tally()
    run.close()
    print(f"  closure {_closure(t):.2e}, alive {t['n_alive']}", flush=True)
    assert t["n_alive"] > 50_000_000
    _check_run_properties(t, None)


def test_fullsize_fp64_delta_rays(P):
    """The 2e7-electron FP64 workload with delta rays (about a million
    records a step): 2000 electrons drawn at step 40 stepped once by the
    oracle against the GPU's step of the whole population (the parents; a
    delta ray's id depends on the whole step's records), then whole-run
    properties: ledger closure, unique ids, no lost delta rays."""
    cfg, srcs, _ = W.config_fp64_large()
    cfg["physics"] |= W.PHYS_DELTA
    cfg["max_particles"] = 30_000_000
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(40)
    st0 = run.get_state()
    run.step(1)
    st1 = run.get_state()
    t = run.tally()
    run.close()
    n0 = len(st0["ids"])
    print(f"  step 40: {n0} electrons alive, {st0['delta_next']} delta rays so far, "
          f"{t['counters']['n_delta']} emitted", flush=True)
    assert st0["delta_next"] > 1_000_000
    pick = np.random.default_rng(5).choice(n0, 2000, replace=False)
    ids = st0["ids"][pick]
    ora = OracleRun(cfg)
    ora.set_state(dict(_subset(st0, ids), step=st0["step"], next_id=st0["next_id"],
                       delta_next=st0["delta_next"]))
    ora.step()
    ref = ora.state()
    born = ref["ids"] >= 0x80000000 + st0["delta_next"]
    ref = {k: (v[~born] if k in ("pos", "p", "w", "tau", "tau_d", "ids") else v) for k, v in ref.items()}
    got = _subset(st1, ids)
    err, only = particle_errors(got, ref, cfg["dx"])
    print(f"  compared {len(err['ids'])}: max|dp|={err['p'].max():.2e} max|dtau_d|={err['tau_d'].max():.2e} "
          f"only-one-side={len(only)}", flush=True)
    assert not only and len(err["ids"]) > 1800
    for k in ("p", "pos", "tau", "tau_d", "w"):
        assert err[k].max() < 1e-10, k
    assert _closure(t) < 1e-6
    assert t["counters"]["n_delta_lost"] == 0
    assert len(np.unique(st1["ids"])) == len(st1["ids"])


def test_fullsize_fp64_urban_scatter(P):
    """The 2e7-electron FP64 workload with the Urban-type scatter: 2000
    electrons drawn at step 30 stepped once by the oracle in the GPU's fields
    against the GPU's step of the whole population, and ledger closure."""
    cfg, srcs, _ = W.config_fp64_large()
    cfg["physics"] |= W.PHYS_URBAN
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(30)
    st0 = run.get_state()
    run.step(1)
    st1 = run.get_state()
    t = run.tally()
    run.close()
    n0 = len(st0["ids"])
    pick = np.random.default_rng(7).choice(n0, 2000, replace=False)
    ids = st0["ids"][pick]
    ora = OracleRun(cfg)
    ora.set_state(dict(_subset(st0, ids), step=st0["step"], next_id=st0["next_id"]))
    ora.step()
    ref = ora.state()
    got = _subset(st1, ids)
    err, only = particle_errors(got, ref, cfg["dx"])
    print(f"  compared {len(err['ids'])}: max|dp|={err['p'].max():.2e} max|dx|/dx={err['pos'].max():.2e} "
          f"only-one-side={len(only)}", flush=True)
    assert not only and len(err["ids"]) > 1800
    for k in ("p", "pos", "tau", "w"):
        assert err[k].max() < 1e-10, k
    assert _closure(t) < 1e-6


def _box_subset(st, lo, hi, dx):
    """Electrons whose start-of-step cell lies in the box [lo, hi)."""
    c = np.floor(st["pos"] / dx).astype(np.int64)
    sel = np.all((c >= lo) & (c < hi), axis=1)
    return {k: (st[k][sel] if k in ("pos", "p", "w", "tau", "tau_d", "ids") else st[k]) for k in st}, int(sel.sum())


def _pick_boxes(st, cfg, cap=1_500_000):
    """Two boxes of cells away from the walls: one around the densest 4^3
    tile (where tiles carry their LDS regions over many chunks) and one
    around a tile drawn at random from the occupied ones; each is shrunk
    until it holds at most `cap` electrons."""
    dx = cfg["dx"]
    dims = np.array([cfg["nx"], cfg["ny"], cfg["nz"]])
    c = np.floor(st["pos"] / dx).astype(np.int64)
    t = c >> 2
    nt = dims // 4
    key = t[:, 0] + nt[0] * (t[:, 1] + nt[1] * t[:, 2])
    u, cnt = np.unique(key, return_counts=True)
    rng = np.random.default_rng(11)
    centres = [u[np.argmax(cnt)], u[rng.integers(len(u))]]
    boxes = []
    for k in centres:
        tc = np.array([k % nt[0], (k // nt[0]) % nt[1], k // (nt[0] * nt[1])]) * 4 + 2
        for half in (8, 6, 5, 4, 3):
            lo = np.maximum(tc - half, 2)
            hi = np.minimum(tc + half, dims - 2)
            n = int(np.sum(np.all((c >= lo) & (c < hi), axis=1)))
            if n <= cap:
                break
        boxes.append((lo, hi, n))
    return boxes


@pytest.mark.parametrize("which,precision,n_pre", [("c2", W.FP64, 30), ("c2", W.FP64, 60),
                                                   ("c2", W.FP32_MIXED, 60), ("c3", W.FP32_MIXED, 25)])
def test_fullsize_grid_parity(P, which, precision, n_pre):
    """Grid side at full size, in the configuration bench.py times.  (1) The
    hot current and collisional heat of the GPU's step of the whole
    population, in two boxes (the densest tile's surroundings and a random
    occupied tile's), against the oracle's step of every electron that
    starts in the box and of the step's injections: j_h on the nodes only
    those electrons reach, heat in the box's cells.  (2) The GPU's j_h and heat fed to the oracle's field
    and heating update from the GPU's start-of-step grid: E, B, Te, Ti and
    eta over the whole grid."""
    if which == "c2":
        cfg, srcs, _ = W.config_fp64_large()
    else:
        cfg, srcs, _ = W.config_mixed_large()
    cfg["precision"] = precision
    fp64 = precision == W.FP64
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(n_pre)
    st0 = run.get_state()
    run.step(1)
    st1 = run.get_state()
    run.close()
    dx = cfg["dx"]
    print(f"  {which} precision {precision} step {n_pre}: {len(st0['ids'])} electrons", flush=True)
    tol_j = 1e-10 if fp64 else 1e-5
    tol_h = 1e-10 if fp64 else 1e-4
    for lo, hi, n in _pick_boxes(st0, cfg):
        sub, n = _box_subset(st0, lo, hi, dx)
        ora = OracleRun(cfg)
        for s in srcs:           # the electrons this step injects (at the front face) heat the box too
            ora.add_source(s)
        ora.set_state(dict(sub, step=st0["step"], next_id=st0["next_id"]))
        ora.step()
        ref = ora.state()
        sl = tuple(slice(lo[d] + 1, hi[d] - 1) for d in range(3))     # nodes [lo+1, hi-2]
        ej = field_rel([g[sl] for g in st1["j"]], [r[sl] for r in ref["j"]])
        cl = tuple(slice(lo[d], hi[d]) for d in range(3))
        eh = rel(st1["ion_heat"][cl], ref["ion_heat"][cl])
        print(f"  box {lo}-{hi}: {n} electrons, j {ej:.2e}, heat {eh:.2e}", flush=True)
        assert n > 1000
        assert ej <= tol_j and eh <= tol_h
    # the oracle's grid update from the GPU's start-of-step grid and this step's j_h and heat
    ora = OracleRun(cfg)
    ora.set_state(dict(pos=np.zeros((0, 3)), p=np.zeros((0, 3)), w=np.zeros(0), tau=np.zeros(0),
                       ids=np.zeros(0, dtype=np.uint32), E=st0["E"], B=st0["B"], Te=st0["Te"],
                       Ti=st0["Ti"], eta=st0["eta"]))
    ora.j = tuple(np.array(x, dtype=np.float64) for x in st1["j"])
    ora.ion_heat = np.array(st1["ion_heat"], dtype=np.float64)
    ora.grid_update()
    s = ora.solid
    tol_f = 1e-10 if fp64 else 1e-5
    errs = dict(E=field_rel(st1["E"], ora.E), B=field_rel(st1["B"], ora.B), Te=rel(st1["Te"][s], ora.Te[s]),
                Ti=rel(st1["Ti"][s], ora.Ti[s]), eta=rel(st1["eta"][s], ora.eta[s]))
    print("  grid update: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["E"] <= tol_f and errs["B"] <= tol_f
    assert errs["Te"] <= 1e-10 and errs["Ti"] <= 1e-10 and errs["eta"] <= 1e-10
