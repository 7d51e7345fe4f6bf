"""Oracle pins for compound solids (App. A): the paper's criterion that two
overlapping halves of one material behave as that material (for every
process of the step), the Bragg mixture rule that the per-element sum of eq.
stop_ion amounts to, a vanishing second element, and the compound
resistivity between its elements'."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleRun
from oracle import constants as K
from oracle import particles as PT
from oracle import run as R
from oracle import solid as S

MEV = 1e6 * K.E
AU = W.MATERIALS["Au"]


def _halves_cfg(**over):
    """Gold as two overlapping solids of half the density each."""
    return dict(rho=AU["rho"] / 2, n_extra=1, extra_Z=(79.0, 0.0, 0.0), extra_A=(AU["A"], 0.0, 0.0),
                extra_rho=(AU["rho"] / 2, 0.0, 0.0), **over)


@pytest.mark.parametrize("phys", [W.PHYS_ALL & ~W.PHYS_FIELDS, (W.PHYS_ALL & ~W.PHYS_FIELDS) | W.PHYS_DELTA])
def test_two_halves_of_one_material_are_that_material(phys):
    """App. A's criterion for its compound heating rule, applied to every
    process: gold as two half-density solids gives the same electrons,
    temperatures and resistivity as gold, step after step (30 steps, all
    collisions, heating, field solve)."""
    base = dict(nx=16, ny=12, nz=12, x_lo=2e-6, x_hi=14e-6, physics=phys, brem_boost=10.0,
                max_particles=40000, series_len=32)
    src = W.source(n_macro=3000, y0=6e-6, z0=6e-6, r_fwhm=4e-6, T_hot=2 * MEV, t_end=0.2e-12)
    runs = []
    for cfg in (W.base_config(**base), W.base_config(**base, **_halves_cfg())):
        r = OracleRun(cfg)
        r.add_source(src)
        r.run(30)
        runs.append(r)
    a, b = runs
    assert a.n_sub == b.n_sub
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["ids"], sb["ids"]) and len(sa["ids"]) > 1000
    assert np.allclose(sb["p"], sa["p"], rtol=1e-11, atol=1e-11 * np.abs(sa["p"]).max())
    assert np.allclose(sb["pos"], sa["pos"], rtol=0, atol=1e-11 * base["nx"] * 1e-6)
    s = a.solid
    assert np.allclose(b.Te[s], a.Te[s], rtol=1e-11)
    assert np.allclose(b.Ti[s], a.Ti[s], rtol=1e-11)
    assert np.allclose(b.eta[s], a.eta[s], rtol=1e-11)
    assert a.Te[s].max() > 2 * W.base_config()["T0"]          # the heating did act


def test_element_sum_of_stop_ion_is_the_bragg_rule():
    """Summing eq. stop_ion over the elements equals the formula for one
    medium with Z n = sum(Z n) and ln I = sum(Z n ln I)/sum(Z n) (Bragg's
    additivity for the mean excitation energy)."""
    pl = W.plastic()
    elems = [dict(S.element(pl["Z"], pl["A"], pl["rho"]), I_ex=11 * K.E * pl["Z"]),
             dict(S.element(1.0, 1.008, pl["extra_rho"][0]), I_ex=11 * K.E)]
    zn = sum(e["Z"] * e["n"] for e in elems)
    lnI = sum(e["Z"] * e["n"] * math.log(e["I_ex"]) for e in elems) / zn
    eps = np.array([0.05, 0.3, 1.0, 5.0, 40.0]) * MEV
    p = np.zeros((len(eps), 3))
    p[:, 2] = PT.momentum_of_energy(eps)
    mix = PT.stopping_ion_mix(eps, p, elems)
    one = PT.stopping_ion(eps, p, 1.0, zn, math.exp(lnI))
    assert np.allclose(mix, one, rtol=1e-12)
    # and the Davies variance likewise with the Z^2 n-weighted screening log
    s2 = PT.davies_sigma2_mix(p, elems, 1e-15)
    ref = sum(PT.davies_sigma2(p, e["Z"], e["n"], 1e-15) for e in elems)
    assert np.allclose(s2, ref, rtol=1e-12)                    # no log clamps at these energies


def test_vanishing_second_element_leaves_the_material():
    """A second element at 1e-12 of the density changes nothing at 1e-9."""
    Te, Ti = np.array([2e4, 3e5, 4e6]), np.array([1.5e4, 2e5, 1e6])
    one = [S.element(79.0, AU["A"], AU["rho"])]
    two = one + [S.element(6.0, 12.011, AU["rho"] * 1e-12)]
    e1, _, _ = S.resistivity_mix(Te, Ti, one, 7.0, 3.5)
    e2, _, _ = S.resistivity_mix(Te, Ti, two, 7.0, 3.5)
    assert np.allclose(e1, e2, rtol=1e-9)
    r1 = S.heat_update_mix(Te, Ti, np.full(3, 1e24), np.full(3, 1e-12), e1, 1e-14, 1e-18, one, 7.0, 3.5)
    r2 = S.heat_update_mix(Te, Ti, np.full(3, 1e24), np.full(3, 1e-12), e2, 1e-14, 1e-18, two, 7.0, 3.5)
    for x, y in zip(r1, r2):
        assert np.allclose(x, y, rtol=1e-9)


def test_compound_resistivity_lies_between_its_elements():
    """sum(x Z* eta)/sum(x Z*) is a weighted mean of the elements' values at
    the total ion density."""
    pl = W.plastic()
    elems = [S.element(pl["Z"], pl["A"], pl["rho"]), S.element(1.0, 1.008, pl["extra_rho"][0])]
    n_t = sum(e["n"] for e in elems)
    T = np.logspace(4, 8, 9)
    eta, _, _ = S.resistivity_mix(T, T, elems, 7.0, 3.5)
    per = [S.resistivity(T, T, e["Z"], e["A"], n_t * e["A"] * K.AMU, 7.0, 3.5)[0] for e in elems]
    lo, hi = np.minimum(*per), np.maximum(*per)
    assert np.all(eta >= lo * (1 - 1e-12)) and np.all(eta <= hi * (1 + 1e-12))
