"""GPU tests of the serving engine: continuous batching gives each run the
bitwise-same result alone and in a mix; admission by footprint; cancelling a
run mid-flight leaves the others unaffected."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_01723_amd as P
    return P


def _reqs():
    """Three small runs with different grids, materials, precisions and seeds."""
    a, sa, _ = W.config_small()
    a.update(precision=W.FP32_MIXED, brem_boost=10.0, sort_every=1, max_particles=3000)
    sa[0]["n_macro"] = 3000
    b = W.base_config(nx=40, ny=20, nz=20, x_lo=4e-6, x_hi=36e-6, material="Cu",
                      precision=W.FP32_MIXED, I0=W.intensity_wcm2(3e21), seed=5, sort_every=2,
                      max_particles=2500, series_len=64)
    sb = [W.source(n_macro=2500, y0=10e-6, z0=10e-6, r_fwhm=4e-6, T_hot=5 * W.MEV)]
    c = W.base_config(nx=24, ny=16, nz=12, x_lo=2e-6, x_hi=20e-6, material="Al",
                      precision=W.FP64, seed=9, max_particles=1500, series_len=64)
    sc = [W.source(n_macro=1500, y0=8e-6, z0=6e-6, r_fwhm=3e-6, T_hot=1 * W.MEV)]
    return [(a, sa, 60), (b, sb, 45), (c, sc, 50)]


def _alone(P, cfg, srcs, steps):
    run = P.Run(cfg)
    for s in srcs:
        run.inject(s)
    run.step(steps)
    t = run.tally()
    st = run.get_state()
    run.close()
    return t, st


def _same(t1, st1, t2, st2):
    o1, o2 = np.argsort(st1["ids"]), np.argsort(st2["ids"])
    assert np.array_equal(st1["ids"][o1], st2["ids"][o2])
    assert np.array_equal(st1["p"][o1], st2["p"][o2])
    assert np.array_equal(st1["pos"][o1], st2["pos"][o2])
    assert np.array_equal(st1["Te"], st2["Te"])
    assert np.array_equal(st1["B"][1], st2["B"][1])
    assert np.array_equal(t1["hist_E"], t2["hist_E"])
    assert t1["ledger"] == t2["ledger"]
    assert t1["step"] == t2["step"]


def test_alone_equals_mixed(P):
    reqs = _reqs()
    alone = [_alone(P, *r) for r in reqs]
    eng = P.Engine(max_runs=8)
    runs = {}
    # staggered admission: run 0 first, run 1 after 7 ticks, run 2 after 20
    runs[0] = eng.admit(*reqs[0])
    eng.step(7)
    runs[1] = eng.admit(*reqs[1])
    eng.step(13)
    runs[2] = eng.admit(*reqs[2])
    assert eng.stats()["resident"] == 3
    finished = {}
    for _ in range(200):
        eng.step(3)
        for r in eng.poll():
            k = [k for k, v in runs.items() if v is r][0]
            finished[k] = (r.tally(), r.get_state())
            eng.retire(r)
        if len(finished) == 3:
            break
    assert len(finished) == 3
    for k in range(3):
        _same(*alone[k], *finished[k])
    eng.close()


def test_admission_by_footprint_and_cancel(P):
    reqs = _reqs()
    fp = [P.footprint(r[0]) for r in reqs]
    eng = P.Engine(hbm_budget=max(fp[0], fp[1]) + fp[2] + 1024, max_runs=8)
    r0 = eng.admit(*reqs[0])
    r2 = eng.admit(*reqs[2])
    assert r0 is not None and r2 is not None
    assert eng.admit(*reqs[1]) is None           # does not fit now
    eng.step(10)
    eng.retire(r0)                               # cancel mid-flight
    r1 = eng.admit(*reqs[1])                     # fits after the slot frees
    assert r1 is not None
    done = {}
    for _ in range(100):
        eng.step(5)
        for r in eng.poll():
            done[id(r)] = (r, r.tally(), r.get_state())
            eng.retire(r)
        if len(done) == 2:
            break
    assert len(done) == 2
    t1, st1 = _alone(P, *reqs[1])
    t2, st2 = _alone(P, *reqs[2])
    got = {d[1]["step"]: d for d in done.values()}
    _same(t2, st2, got[50][1], got[50][2])
    _same(t1, st1, got[45][1], got[45][2])
    eng.close()


def test_serving_loop_small_scan(P):
    """The continuous-batching driver on a shrunken 8-run scan."""
    from paper_2107_01723_amd import serve
    reqs = W.scan_runs(8, seed=3, rate_hz=50.0, scale=0.01)
    out = serve.run_scan(reqs, ticks_per_poll=4)
    assert out["runs"] == 8
    assert out["p99_s"] >= out["p50_s"] > 0
    for i, res in out["results"].items():
        assert res["step"] == reqs[i]["steps"]


def test_delta_run_alone_equals_mixed(P):
    """A run with delta rays batched with runs without them (same precision,
    so one launch serves both kinds): every run bitwise as alone, the delta
    rays and their optical depths included."""
    reqs = _reqs()
    d = W.base_config(nx=24, ny=16, nz=16, x_lo=2e-6, x_hi=22e-6, precision=W.FP64, seed=4,
                      brem_boost=10.0, physics=W.PHYS_ALL | W.PHYS_DELTA, sort_every=2,
                      max_particles=20000, series_len=64)
    sd = [W.source(n_macro=1500, y0=8e-6, z0=8e-6, r_fwhm=4e-6, T_hot=2 * W.MEV)]
    mix = [reqs[2], (d, sd, 40), reqs[0]]
    alone = [_alone(P, *r) for r in mix]
    assert alone[1][0]["counters"]["n_delta"] > 100
    eng = P.Engine(max_runs=8)
    runs = {k: eng.admit(*r) for k, r in enumerate(mix)}
    finished = {}
    for _ in range(200):
        eng.step(3)
        for r in eng.poll():
            k = [k for k, v in runs.items() if v is r][0]
            finished[k] = (r.tally(), r.get_state())
            eng.retire(r)
        if len(finished) == 3:
            break
    assert len(finished) == 3
    for k in range(3):
        _same(*alone[k], *finished[k])
    o1, o2 = np.argsort(alone[1][1]["ids"]), np.argsort(finished[1][1]["ids"])
    assert np.array_equal(alone[1][1]["tau_d"][o1], finished[1][1]["tau_d"][o2])
    assert alone[1][0]["counters"] == finished[1][0]["counters"]
    eng.close()


def test_scan_smallest_runs_against_oracle(P):
    """The two smallest runs of the 64-run scan (the bench's request stream),
    served by the engine beside two larger ones: after 40 steps (inside the
    1 ps injection) each one's state is taken, the oracle steps it once
    (with that step's injections) and the engine's next step of the batch
    matches it per electron within 1e-5 (FP32-mixed), electrons whose
    discrete path differs counted (<= 0.5 %)."""
    from oracle import OracleRun
    from parity_util import particle_errors
    reqs = W.scan_runs(64, seed=0)
    size = [r["srcs"][0]["n_macro"] * r["cfg"]["nx"] * r["cfg"]["ny"] * r["cfg"]["nz"] for r in reqs]
    order = np.argsort(size)
    small, big = [int(k) for k in order[:2]], [int(order[len(order) // 2]), int(order[len(order) // 2 + 1])]
    eng = P.Engine(max_runs=8)
    runs = {k: eng.admit(reqs[k]["cfg"], reqs[k]["srcs"], reqs[k]["steps"]) for k in small + big}
    assert all(r is not None for r in runs.values())
    eng.step(40)
    st0 = {k: runs[k].get_state() for k in small}
    eng.step(1)
    for k in small:
        cfg, src = reqs[k]["cfg"], reqs[k]["srcs"][0]
        st1 = runs[k].get_state()
        ora = OracleRun(cfg)
        ora.add_source(src)
        ora.set_state(dict(st0[k]))
        ora.step()
        err, only = particle_errors(st1, ora.state(), cfg["dx"])
        tol = 1e-5
        bad = (err["p"] > tol) | (err["pos"] > tol) | (err["tau"] > tol)
        nflip = int(np.sum(bad)) + len(only)
        print(f"  scan run {k} ({cfg['nx']}x{cfg['ny']}x{cfg['nz']}, {src['n_macro']} electrons scheduled): "
              f"{len(err['ids'])} compared, max|dp|={err['p'][~bad].max():.2e} "
              f"max|dx|/dx={err['pos'][~bad].max():.2e} flips={nflip}", flush=True)
        assert len(err["ids"]) > 10_000
        assert nflip <= 0.005 * len(err["ids"]), (nflip, only[:10])
        assert err["w"].max() <= tol
    eng.close()
