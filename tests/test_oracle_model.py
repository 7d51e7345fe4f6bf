"""Oracle pins for the paper's energy-partition model (Sec. III.B): the
three macro-electrons against the exponential's moments, the integrator
against closed-form paths for each stopping power alone, energy
conservation over the intensity-Z plane, and the dominant mechanisms the
paper reports."""
import math

import numpy as np
import pytest
from scipy import integrate as SI

import workloads as W
from oracle import constants as K
from oracle import model as M
from oracle import particles as PT

MEV = 1e6 * K.E
MEC2 = K.MEC2


def test_macro_electrons_are_the_exponential_moments():
    """Weights sum to N and energies to N T; each bin's mean energy lies in
    the bin; an escape energy below the threshold empties the emitting bin."""
    T, N = 3.1 * MEV, 1e12
    W_, E = M.macro_electrons(T, 1 * MEV, 8.6 * MEV, N)
    assert W_.sum() == pytest.approx(N, rel=1e-14)
    assert E.sum() == pytest.approx(N * T, rel=1e-14)
    mean = E / W_
    assert mean[0] < 1 * MEV <= mean[1] < 8.6 * MEV <= mean[2]
    # the escaping electrons' mean is e_esc + T (memoryless tail)
    assert mean[2] == pytest.approx(8.6 * MEV + T, rel=1e-12)
    W2, E2 = M.macro_electrons(0.2 * MEV, 1 * MEV, 0.5 * MEV, N)
    assert W2[1] == 0.0 and E2[1] == 0.0 and W2.sum() == pytest.approx(N, rel=1e-14)


def _p(**over):
    """A parameter set with every stopping power off (n_i = 0 switches off
    the ionisation) unless given."""
    p = dict(k_brem=0.0, e_th=1 * MEV, Z=1.0, n_i=0.0, I_ex=11 * K.E, s_tnsa=0.0, k_field=0.0,
             tan_c=math.tan(math.radians(20.0)), r_half=2.5e-6)
    p.update(over)
    return {k: np.atleast_1d(np.float64(v)) for k, v in p.items()}


def test_brem_alone_is_exponential_and_its_photon_part_closed_form():
    """dE/dx = -k (1 + E/mc^2): the path to rest is (mc^2/k) ln(1 + E0/mc^2);
    the part above the threshold, k (1 + (E - E_th)/mc^2) for E > E_th, takes
    (E0 - E_th) - E_th ln((mc^2 + E0)/(mc^2 + E_th))."""
    k = 2.0 * MEV / 1e-3
    e0, eth = 20 * MEV, 1 * MEV
    loss, left = M.integrate(np.array([e0]), _p(k_brem=k), 4000, np.array([np.inf]))
    assert loss[0, 0] == pytest.approx(e0, rel=1e-12)                  # all of it radiated
    thr = (e0 - eth) - eth * math.log((MEC2 + e0) / (MEC2 + eth))
    assert loss[1, 0] == pytest.approx(thr, rel=1e-6)
    # the path: stop the integration at a depth and compare the energy left
    x_stop = 0.5 * (MEC2 / k) * math.log(1 + e0 / MEC2)
    _, left = M.integrate(np.array([e0]), _p(k_brem=k), 4000, np.array([x_stop]))
    expect = (e0 + MEC2) * math.exp(-k * x_stop / MEC2) - MEC2
    assert left[0] == pytest.approx(expect, rel=1e-6)


def test_reflux_alone_is_linear():
    """Constant stopping: the energy left at depth x is E0 - S x."""
    s = 0.7 * MEV / 1e-4
    e0 = 5 * MEV
    _, left = M.integrate(np.array([e0]), _p(s_tnsa=s), 4000, np.array([3e-4]))
    assert left[0] == pytest.approx(e0 - s * 3e-4, rel=1e-9)
    loss, _ = M.integrate(np.array([e0]), _p(s_tnsa=s), 4000, np.array([np.inf]))
    assert loss[3, 0] == pytest.approx(e0, rel=1e-12)


def test_field_alone_matches_its_closed_form():
    """dE/dx = -C/(x t + r)^2: E(x) = E0 - (C/t)(1/r - 1/(x t + r))."""
    C, t, r = 2e-19, math.tan(math.radians(20.0)), 2.5e-6
    e0, L = 30 * MEV, 1e-4
    _, left = M.integrate(np.array([e0]), _p(k_field=C, tan_c=t, r_half=r), 4000, np.array([L]))
    expect = e0 - (C / t) * (1.0 / r - 1.0 / (L * t + r))
    assert expect > 0
    assert left[0] == pytest.approx(expect, rel=1e-7)


def test_ionisation_path_is_the_range_integral():
    """Ionisation plus a weak constant loss: the depth reached when all the
    energy is spent is the integral of dE / (S_ion + s)."""
    n_i = 6e28
    s = 0.01 * MEV / 1e-4
    p = _p(Z=79.0, n_i=n_i, I_ex=11 * K.E * 79, s_tnsa=s)
    e0 = 2 * MEV

    def inv(e):
        mom = np.array([[PT.momentum_of_energy(e), 0.0, 0.0]])
        return 1.0 / (PT.stopping_ion(np.array([e]), mom, 79.0, n_i, 11 * K.E * 79)[0] + s)

    rng = SI.quad(inv, 0.0, e0, limit=400, points=[1e3 * K.E, 1e4 * K.E])[0]
    _, left = M.integrate(np.array([e0]), p, 4000, np.array([0.5 * rng]))
    # half the range: the energy left is where the remaining range is half
    rest = SI.quad(inv, 0.0, left[0], limit=400, points=[1e3 * K.E, 1e4 * K.E])[0]
    assert rest == pytest.approx(0.5 * rng, rel=1e-5)
    loss, _ = M.integrate(np.array([e0]), p, 4000, np.array([np.inf]))
    assert loss[2, 0] + loss[3, 0] == pytest.approx(e0, rel=1e-12)
    assert loss[3, 0] == pytest.approx(s * rng, rel=1e-5)


def test_energy_is_conserved_over_the_plane():
    """Over the intensity-Z plane every injected joule goes to exactly one of
    brem, ionisation, reflux, field or escape (photons above the threshold
    are part of brem)."""
    m = W.model_inputs()
    I, Z = W.model_scan_grid(n_int=5, z_values=[1, 6, 13, 29, 47, 79, 92])
    f = M.partition(m, I, Z, 1000)
    # to the integration's accuracy (the losses sum to Simpson's rule for the energy)
    assert np.allclose(f[0] + f[2] + f[3] + f[4] + f[5], 1.0, rtol=0, atol=1e-9)
    assert np.all(f >= 0.0) and np.all(f[1] <= f[0])


def test_dominant_mechanisms_as_the_paper_reports():
    """Sec. III.B: for high Z, ionisation dominates at low intensity and
    bremsstrahlung at high intensity; for low Z at high intensity, reflux
    dominates."""
    m = W.model_inputs()
    I = W.intensity_wcm2(np.array([1e20, 1e22, 1e22]))
    Z = np.array([79.0, 79.0, 13.0])
    f = M.partition(m, I, Z, m["nsteps"])
    dom = [("brem", "ionisation", "reflux", "field", "escaped")[k]
           for k in np.argmax(f[[0, 2, 3, 4, 5]], axis=0)]
    assert dom == ["ionisation", "brem", "reflux"]
    # and eta_e->gamma rises with intensity and with Z
    assert f[1, 1] > f[1, 0] and f[1, 1] > f[1, 2]
