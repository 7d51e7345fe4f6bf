"""Oracle pins for the bremsstrahlung enhancement by background ionisation,
eq. F_sigma (Sec. II.B): its limits, its screening logarithm against the
fine-structure constant, and its use in the step (both the emission depth
and the sub-cut loss of the electron's start-of-step cell scale by it)."""
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


def test_screening_log_is_complete_screening_log():
    """ln(a_s m_e c / hbar) with a_s = 1.4 a_B Z^-1/3 equals ln(1.4/alpha Z^-1/3),
    the logarithm of the complete-screening bremsstrahlung prefactor: the
    Bohr radius is the reduced Compton wavelength over alpha."""
    for Z in (13.0, 29.0, 79.0):
        a_s = 1.4 * K.A_BOHR * Z ** (-1.0 / 3.0)
        assert math.log(a_s * K.ME * K.C / K.HBAR) == pytest.approx(
            math.log(1.4 / K.ALPHA * Z ** (-1.0 / 3.0)), rel=1e-12)


def test_f_sigma_is_one_when_debye_length_equals_screening_length():
    Z, A, rho = AU["Z"], AU["A"], AU["rho"]
    n_i = S.ion_density(rho, A)
    a_s = 1.4 * K.A_BOHR * Z ** (-1.0 / 3.0)
    for Te in (1e5, 1e6, 1e7):
        Zs = float(S.zstar_more(Z, A, rho, Te))
        Ti = a_s ** 2 * Zs ** 2 * K.E ** 2 * n_i / (K.EPS0 * K.KB)   # lambda_D = a_s
        assert float(S.f_sigma(Te, Ti, Z, A, rho)) == pytest.approx(1.0, abs=1e-12)


def test_f_sigma_fully_ionised_is_ratio_of_screening_logs():
    """Z* -> Z: F = ln(lambda_D / lbar_C) / ln(a_s / lbar_C)."""
    Z, A, rho = AU["Z"], AU["A"], AU["rho"]
    n_i = S.ion_density(rho, A)
    Te = Ti = 1e10
    Zs = float(S.zstar_more(Z, A, rho, Te))
    assert Zs / Z > 0.999
    lam = math.sqrt(K.EPS0 * K.KB * Ti / (Zs ** 2 * K.E ** 2 * n_i))
    lbar = K.HBAR / (K.ME * K.C)
    a_s = 1.4 * K.A_BOHR * Z ** (-1.0 / 3.0)
    ratio = math.log(lam / lbar) / math.log(a_s / lbar)
    # the ratio holds exactly at Z* = Z; the departure is (1 - (Z*/Z)^2) times
    # the log quotient
    bound = abs(math.log(lam / a_s) / math.log(a_s / lbar)) * (1 - (Zs / Z) ** 2) + 1e-12
    assert abs(float(S.f_sigma(Te, Ti, Z, A, rho)) - ratio) <= bound


def test_f_sigma_cold_solid_is_near_one_and_monotone_in_ion_temperature():
    """A cold solid is weakly ionised, so (Z*/Z)^2 keeps F near 1; a hotter
    ion population has a longer Debye length and a larger F."""
    Z, A, rho = AU["Z"], AU["A"], AU["rho"]
    T0 = 11604.5
    assert abs(float(S.f_sigma(T0, T0, Z, A, rho)) - 1.0) < 0.02
    Ti = np.logspace(4, 8, 9)
    f = S.f_sigma(np.full_like(Ti, 1e6), Ti, Z, A, rho)
    assert np.all(np.diff(f) > 0)


def test_step_scales_emission_depth_and_subcut_loss_by_f_sigma():
    """One oracle step of electrons in one hot cell, brem only: the drop of
    the optical depth and the sub-cut loss are F_sigma of that cell times
    their values without the enhancement."""
    cfg = W.base_config(nx=8, ny=8, nz=8, x_lo=0.0, x_hi=8e-6, brem_boost=1.0,
                        physics=R.PHYS_BREM, max_particles=16, series_len=4)
    n = 6
    pos = np.array([[3.5e-6, 4.2e-6, 2.7e-6]] * n)
    eps = np.linspace(1, 30, n) * MEV
    p = np.column_stack([np.zeros(n), np.zeros(n), [PT.momentum_of_energy(e) for e in eps]])
    base = dict(pos=pos, p=p, w=np.ones(n), tau=np.full(n, 50.0), ids=np.arange(n, dtype=np.uint32))
    out = {}
    for phys in (R.PHYS_BREM, R.PHYS_BREM | R.PHYS_FSIGMA):
        r = OracleRun(dict(cfg, physics=phys))
        Te, Ti = r.Te.copy(), r.Ti.copy()
        Te[3, 4, 2], Ti[3, 4, 2] = 3e6, 8e6
        r.set_state(dict(base, Te=Te, Ti=Ti))
        r.step()
        out[phys] = (50.0 - r.tau, r.ledger["rad_subcut"])
    F = float(S.f_sigma(3e6, 8e6, cfg["Z"], cfg["A"], cfg["rho"]))
    assert abs(F - 1.0) > 1e-3
    d0, s0 = out[R.PHYS_BREM]
    d1, s1 = out[R.PHYS_BREM | R.PHYS_FSIGMA]
    assert np.allclose(d1, F * d0, rtol=1e-12)
    assert s1 == pytest.approx(F * s0, rel=1e-9)
