"""GPU parity of the Urban-type elastic scatter (App. B: model functions
matched to the Lewis moments) against the FP64 oracle: whole runs without
field feedback, one step with every field on, FP32-mixed one step, the
depth-dose benchmark setup with this model, and a batch that mixes it with
Davies runs."""
import numpy as np
import pytest

import workloads as W
from oracle import OracleRun

from parity_util import field_rel, gpu_from_oracle, oracle_at, particle_errors, rel, small_config

pytestmark = pytest.mark.gpu

URBAN_PHYS = (W.PHYS_ALL & ~W.PHYS_FIELDS) | W.PHYS_URBAN


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_01723_amd as P
    P.check_abi()
    return P


@pytest.mark.parametrize("sort_every,extra", [(0, 0), (3, W.PHYS_DELTA)])
def test_urban_whole_run_fp64(P, sort_every, extra):
    """40 steps of injection with collisions and the Urban-type scatter,
    field feedback off (electrons independent), with and without the tile
    sort, alone and with delta rays: every electron, the counts and the
    ledger."""
    cfg, srcs, _ = small_config(6000, brem_boost=10.0, physics=URBAN_PHYS | extra, sort_every=sort_every,
                                max_particles=60000)
    ora = oracle_at(cfg, srcs, 40)
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(40)
    t = run.tally()
    st, ref = run.get_state(), ora.state()
    err, only = particle_errors(st, ref, cfg["dx"])
    back = float(np.mean(ref["p"][:, 0] < 0))
    print(f"  alive {len(err['ids'])}, max|dp| {err['p'].max():.2e}, max|dx|/dx {err['pos'].max():.2e}, "
          f"moving back {back:.3f}", flush=True)
    assert not only, only[:10]
    assert len(err["ids"]) > 1500
    for k in ("p", "pos", "tau", "w"):
        assert err[k].max() < 1e-10, (k, err[k].max())
    for k in ("n_injected", "n_emitted", "n_reflux", "n_escaped", "n_stopped", "n_delta"):
        assert t["counters"][k] == ora.counters[k], k
    for k in ("injected", "ionisation", "rad_discrete", "reflux", "stopped", "escaped", "photon_thr"):
        assert t["ledger"][k] == pytest.approx(ora.ledger[k], rel=1e-8, abs=1e-12 * ora.ledger["injected"]), k
    run.close()


def test_urban_one_step_fields_on(P):
    """Every process and the field feedback on, one step from an identical
    state at step 50: electrons, E, B, Te."""
    cfg, srcs, _ = small_config(10000, brem_boost=10.0, physics=W.PHYS_ALL | W.PHYS_URBAN)
    ora = oracle_at(cfg, srcs, 50)
    run = gpu_from_oracle(P, cfg, srcs, ora)
    ora.step()
    run.step(1)
    got, ref = run.get_state(), ora.state()
    err, only = particle_errors(got, ref, cfg["dx"])
    assert not only
    assert err["p"].max() < 1e-10 and err["pos"].max() < 1e-10
    assert field_rel(got["E"], ref["E"]) < 1e-9 and field_rel(got["B"], ref["B"]) < 1e-9
    s = ora.solid
    assert rel(got["Te"][s], ref["Te"][s]) < 1e-10
    run.close()


def test_urban_fp32_one_step(P):
    """FP32-mixed from the oracle's FP64 state at step 60: per electron 1e-5
    (the model's parameters are solved in FP64 in both precisions), flipped
    discrete decisions <= 0.1 %."""
    cfg, srcs, _ = small_config(10000, precision=W.FP32_MIXED, brem_boost=10.0, physics=URBAN_PHYS)
    ora = oracle_at(cfg, srcs, 60)
    run = gpu_from_oracle(P, cfg, srcs, ora)
    ora.step()
    run.step(1)
    err, only = particle_errors(run.get_state(), ora.state(), cfg["dx"])
    bad = (err["p"] > 1e-5) | (err["pos"] > 1e-5) | (err["tau"] > 1e-5)
    nflip = int(np.sum(bad)) + len(only)
    print(f"  n={len(err['ids'])} max|dp| of the rest {err['p'][~bad].max():.2e} flips {nflip}", flush=True)
    assert len(err["ids"]) > 1500
    assert nflip <= 1e-3 * len(err["ids"])
    run.close()


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_depth_dose_with_urban_scatter(P, precision):
    """The depth-dose benchmark setup of App. C with the Urban-type model
    in place of Davies through its 2 ps: FP64 every electron, every cell's
    temperature, the counts and the ledger; FP32-mixed the depth-dose profile
    and the counts within FP32 tolerances."""
    cfg, beam, steps = W.config_depth_dose(urban=True)
    cfg["precision"] = precision
    ora = OracleRun(cfg)
    ora.add_beam(beam)
    run = P.Run(cfg)
    run.inject_beam(beam)
    ora.run(steps)
    run.step(steps)
    t, st, ref = run.tally(), run.get_state(), ora.state()
    prof_g = (st["Te"] - cfg["T0"]).sum(axis=(1, 2))
    prof_r = (ref["Te"] - cfg["T0"]).sum(axis=(1, 2))
    l1 = np.sum(np.abs(prof_g - prof_r)) / np.sum(np.abs(prof_r))
    print(f"  escaped {t['counters']['n_escaped']} / {ora.counters['n_escaped']}, stopped "
          f"{t['counters']['n_stopped']} / {ora.counters['n_stopped']}, profile L1 {l1:.2e}", flush=True)
    assert ora.counters["n_escaped"] > 500 and ora.counters["n_stopped"] > 500
    if precision == W.FP64:
        assert t["counters"]["n_escaped"] == ora.counters["n_escaped"]
        assert t["counters"]["n_stopped"] == ora.counters["n_stopped"]
        assert rel(st["Te"], ref["Te"]) < 1e-10
        assert l1 < 1e-8
        for k in ("injected", "ionisation", "stopped", "escaped"):
            assert t["ledger"][k] == pytest.approx(ora.ledger[k], rel=1e-9), k
    else:
        dl = {k: abs(t["ledger"][k] - ora.ledger[k]) / abs(ora.ledger[k]) for k in ("injected", "ionisation", "escaped")}
        print("  FP32 ledger rel " + " ".join(f"{k} {v:.1e}" for k, v in dl.items()), flush=True)
        assert abs(t["counters"]["n_escaped"] - ora.counters["n_escaped"]) <= 0.01 * 3200
        assert l1 < 2e-3
        for k in ("injected", "ionisation", "escaped"):
            assert t["ledger"][k] == pytest.approx(ora.ledger[k], rel=1e-4), k
    run.close()


def test_urban_and_davies_runs_in_one_batch(P):
    """A Urban-type run served in the same launches as a Davies run of the
    same precision: each bitwise as alone."""
    cfg_a, srcs, _ = small_config(3000, brem_boost=10.0, physics=W.PHYS_ALL, max_particles=20000)
    cfg_b = dict(cfg_a, physics=W.PHYS_ALL | W.PHYS_URBAN)

    def alone(cfg):
        run = P.Run(cfg)
        run.inject(srcs[0])
        run.step(30)
        st = run.get_state()
        run.close()
        return st

    ref = [alone(cfg_a), alone(cfg_b)]
    eng = P.Engine(max_runs=4)
    runs = [eng.admit(cfg_a, srcs, 30), eng.admit(cfg_b, srcs, 30)]
    done = {}
    for _ in range(100):
        eng.step(3)
        for r in eng.poll():
            done[runs.index(r)] = r.get_state()
            eng.retire(r)
        if len(done) == 2:
            break
    assert len(done) == 2
    for k in range(2):
        o1, o2 = np.argsort(ref[k]["ids"]), np.argsort(done[k]["ids"])
        assert np.array_equal(ref[k]["ids"][o1], done[k]["ids"][o2])
        assert np.array_equal(ref[k]["p"][o1], done[k]["p"][o2])
        assert np.array_equal(ref[k]["Te"], done[k]["Te"])
    # the two models did differ
    assert not np.array_equal(ref[0]["p"][:10], ref[1]["p"][:10])
    eng.close()


def test_urban_on_a_compound_fp64(P):
    """The Urban-type scatter on the CH plastic slab (two elements: the
    transport depths summed over them), 30 steps with collisions and field
    feedback off: every electron against the oracle."""
    cfg, srcs, _ = small_config(4000, brem_boost=10.0, physics=URBAN_PHYS, max_particles=20000, **W.plastic())
    ora = oracle_at(cfg, srcs, 30)
    run = P.Run(cfg)
    run.inject(srcs[0])
    run.step(30)
    err, only = particle_errors(run.get_state(), ora.state(), cfg["dx"])
    print(f"  alive {len(err['ids'])}, max|dp| {err['p'].max():.2e}", flush=True)
    assert not only and len(err["ids"]) > 500
    for k in ("p", "pos", "tau"):
        assert err[k].max() < 1e-10, (k, err[k].max())
    run.close()
