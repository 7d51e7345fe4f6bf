"""Oracle pins for the depth-dose benchmark setup (App. C): the
mono-energetic normal-incidence beam, the open, mirror and periodic
boundary kinds, the continuous-slowing-down range of a beam without scatter
against the integral of 1/S, and the lateral uniformity the periodic and
mirror walls keep."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W
from oracle import OracleRun
from oracle import constants as K
from oracle import particles as PT
from oracle import run as R
from oracle import solid as S

MEV = 1e6 * K.E


def _run(**over):
    cfg, beam, steps = W.config_depth_dose()
    cfg.update(over)
    r = OracleRun(cfg)
    return r, cfg, beam, steps


def test_beam_injection():
    """per_cell electrons in every front-face cell, all at the beam energy
    along +x, positions uniform over each cell's face, ids cell by cell."""
    r, cfg, beam, _ = _run()
    beam = dict(beam, per_cell=400)
    r.add_beam(beam)
    r.step()
    n = 400 * cfg["ny"] * cfg["nz"]
    assert r.counters["n_injected"] == n
    assert r.ledger["injected"] == pytest.approx(n * beam["energy"] * beam["weight"], rel=1e-12)
    # injected at x = 0 with momentum (p, 0, 0): one step of straight flight
    ids = r.ids.astype(np.int64)
    assert np.array_equal(ids, np.arange(n))
    cell = ids // 400
    assert np.array_equal(np.floor(r.X[:, 1]).astype(int), cell % cfg["ny"])
    assert np.array_equal(np.floor(r.X[:, 2]).astype(int), cell // cfg["ny"])
    assert stats.kstest(r.X[:, 1] % 1.0, "uniform").pvalue > 1e-3
    assert np.allclose(r.p[:, 1:], 0.0)


def test_open_and_mirror_boundaries():
    """A mirror wall reflects the position and the normal momentum and
    changes nothing else; an open face lets every electron escape, however
    slow (a reflux face would turn a slow one back)."""
    r, cfg, _, _ = _run(physics=0, bc_x=W.BC_OPEN, bc_y=W.BC_MIRROR, bc_z=W.BC_MIRROR)
    dx = cfg["dx"]
    pos = np.array([[100.5, 0.2, 4.5], [100.5, 7.9, 4.5], [0.1, 4.0, 4.0]]) * dx
    p0 = PT.momentum_of_energy(np.array([1.0, 1.0, 0.05]) * MEV)
    p = np.array([[0.3, -0.9, 0.1], [0.2, 0.95, -0.1], [-1.0, 0.0, 0.0]])
    p = p / np.linalg.norm(p, axis=1)[:, None] * p0[:, None]
    r.set_state(dict(pos=pos, p=p, w=np.ones(3), tau=np.full(3, 30.0), ids=np.arange(3, dtype=np.uint32)))
    e0 = PT.kinetic(p)
    r.step()
    assert r.counters["n_escaped"] == 1 and r.counters["n_reflux"] == 0
    assert r.ledger["escaped"] == pytest.approx(e0[2], rel=1e-12)
    a = r.alive
    assert np.allclose(np.linalg.norm(r.p[a], axis=1), p0[:2], rtol=1e-15)
    assert r.p[0, 1] > 0 and r.p[1, 1] < 0                      # flipped toward the inside
    assert np.allclose(r.p[:2, [0, 2]], p[:2, [0, 2]], rtol=1e-15)
    v = p[:2] / (PT.gamma_of(p[:2]) * K.ME)[:, None]
    y_free = pos[:2, 1] / dx + v[:, 1] * cfg["dt"] / dx
    assert np.allclose(r.X[:2, 1], [-y_free[0], 2 * cfg["ny"] - y_free[1]], rtol=0, atol=1e-12)
    assert r.ledger["reflux"] == 0.0


def test_range_without_scatter_is_the_csda_range():
    """Ionisation only: every electron of the beam runs straight and stops
    (below e_min) at the continuous-slowing-down range, the integral of
    dE / S(E) from e_min to the beam energy (S of eq. stop_ion), within the
    last step's flight and the explicit step's O(dt) error."""
    dx = 150e-6 / 256
    r, cfg, beam, _ = _run(physics=R.PHYS_ION, nx=512, x_hi=512 * dx)   # deeper than the range
    r.add_beam(dict(beam, per_cell=2))
    last = None
    while True:
        r.step()
        a = r.alive
        if not np.any(a):
            break
        last = r.X[a, 0].max() * cfg["dx"]
        assert r.step_index < 2000
    Z, A, rho = cfg["Z"], cfg["A"], cfg["rho"]
    n_i = S.ion_density(rho, A)
    I_ex = 11.0 * K.E * Z

    def inv_S(e):
        p = np.array([[PT.momentum_of_energy(e), 0.0, 0.0]])
        return 1.0 / PT.stopping_ion(np.array([e]), p, Z, n_i, I_ex)[0]

    rng_csda = integrate.quad(inv_S, cfg["e_min"], beam["energy"], limit=200)[0]
    v_min = K.C * math.sqrt(1 - 1 / (1 + cfg["e_min"] / K.MEC2) ** 2)
    print(f"  CSDA range {rng_csda * 1e6:.2f} um, last x {last * 1e6:.2f} um")
    assert abs(last - rng_csda) < v_min * cfg["dt"] + 0.01 * rng_csda
    assert r.counters["n_stopped"] == 2 * cfg["ny"] * cfg["nz"]


def test_periodic_walls():
    """A periodic wall: the electron re-enters through the opposite wall at
    the position a free flight gives modulo the width, with its momentum and
    energy unchanged and nothing booked; periodic x and periodic walls with
    field feedback are refused."""
    r, cfg, _, _ = _run(physics=0)
    dx, ny, nz = cfg["dx"], cfg["ny"], cfg["nz"]
    pos = np.array([[100.5, 0.2, 4.5], [100.5, 7.9, 7.95], [50.0, 3.0, 0.05]]) * dx
    p0 = PT.momentum_of_energy(np.array([1.0, 0.3, 2.0]) * MEV)
    p = np.array([[0.3, -0.9, 0.1], [0.2, 0.95, 0.3], [0.5, 0.1, -0.8]])
    p = p / np.linalg.norm(p, axis=1)[:, None] * p0[:, None]
    r.set_state(dict(pos=pos, p=p, w=np.ones(3), tau=np.full(3, 30.0), ids=np.arange(3, dtype=np.uint32)))
    r.step()
    assert r.counters["n_escaped"] == 0 and r.counters["n_reflux"] == 0
    assert np.array_equal(r.p, p)
    v = p / (PT.gamma_of(p) * K.ME)[:, None]
    free = pos / dx + v * cfg["dt"] / dx
    want = free.copy()
    want[:, 1] = np.mod(free[:, 1], ny)
    want[:, 2] = np.mod(free[:, 2], nz)
    assert np.allclose(r.X, want, rtol=0, atol=1e-12)
    assert r.X[0, 1] > ny - 3 and r.X[1, 1] < 3 and r.X[2, 2] > nz - 3      # they did wrap
    assert r.ledger["reflux"] == 0.0 and r.ledger["escaped"] == 0.0
    with pytest.raises(ValueError):
        _run(bc_x=W.BC_PERIODIC)
    with pytest.raises(ValueError):
        _run(physics=R.PHYS_FIELDS)


@pytest.mark.parametrize("wall", [W.BC_PERIODIC, W.BC_MIRROR])
def test_walls_keep_a_uniform_beam_uniform(wall):
    """With Davies scatter the beam spreads, but periodic or mirror walls on
    a laterally uniform beam keep it uniform in y and z (a wrong wrap or
    reflection piles electrons at a wall)."""
    r, cfg, beam, _ = _run(physics=R.PHYS_ION | R.PHYS_SCATTER, bc_y=wall, bc_z=wall)
    r.add_beam(dict(beam, per_cell=60))
    r.run(60)
    a = r.alive
    assert np.sum(a) > 1000
    for d, n in ((1, cfg["ny"]), (2, cfg["nz"])):
        assert stats.kstest(r.X[a, d] / n, "uniform").pvalue > 1e-3
    # and the scatter did turn them
    assert np.mean(np.abs(r.p[a, 1]) / np.linalg.norm(r.p[a], axis=1)) > 0.2
