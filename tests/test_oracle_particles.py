"""Oracle pins for the particle side: Boris push, collisions, photon angles,
injection samplers, reflux and escape.  Each pin is a closed form, a
textbook formula written independently of the paper's, or a number the
paper prints."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W
from oracle import OracleRun
from oracle import constants as K
from oracle import particles as PT
from oracle import run as R

MEV = 1e6 * K.E


def _one_particle_run(pos, p, phys, nx=32, **over):
    cfg = W.base_config(nx=nx, ny=nx, nz=nx, x_lo=0.0, x_hi=nx * 1e-6, physics=phys,
                        max_particles=64, series_len=8, **over)
    r = OracleRun(cfg)
    pos = np.atleast_2d(pos)
    p = np.atleast_2d(p)
    n = len(pos)
    r.set_state(dict(pos=pos, p=p, w=np.ones(n), tau=np.full(n, 50.0),
                     ids=np.arange(n, dtype=np.uint32)))
    return r


def test_a0_and_escape_energy_match_printed(golden_dir):
    nums = json.load(open(os.path.join(golden_dir, "paper_numbers.json")))
    assert PT.a0_of(1e24, 1e-6) == pytest.approx(nums["a0_at_1e20_Wcm2_1um"]["value"], rel=1e-12)
    # the 86 MeV spectral break at 1e22 W/cm^2 is the escape energy kappa_esc a0 m c^2
    e_esc = nums["kappa_esc"]["value"] * PT.a0_of(1e26, 1e-6) * K.MEC2 / MEV
    assert e_esc == pytest.approx(nums["escape_break_MeV_at_1e22"]["value"], rel=0.02)


def test_boris_gyration_closed_form():
    """Uniform B, E = 0: the rotation per step is exactly 2 atan(Omega dt/2)
    with Omega = e B/(gamma m); |p| is conserved; the discrete orbit lies on a
    circle of radius (v dt/2)/sin(theta/2)."""
    Bz = 800.0
    p0 = PT.momentum_of_energy(1.0 * MEV)
    r = _one_particle_run([16.3e-6, 16.1e-6, 16.0e-6], [p0, 0.0, 0.0], R.PHYS_FIELDS)
    shape = r.B[2].shape
    r.B = (np.zeros(shape), np.zeros(shape), np.full(shape, Bz))
    g = math.sqrt(1 + (p0 / (K.ME * K.C)) ** 2)
    theta = 2 * math.atan(K.E * Bz / (g * K.ME) * r.dt / 2)
    xs = []
    ang0 = math.atan2(r.p[0, 1], r.p[0, 0])
    for n in range(12):
        r.step()
        xs.append(r.pos[0, :2].copy())
        ang = math.atan2(r.p[0, 1], r.p[0, 0])
        # electron (q < 0) in +z field turns counter-clockwise
        dang = (ang - ang0 + math.pi) % (2 * math.pi) - math.pi
        assert dang == pytest.approx((n + 1) * theta - (2 * math.pi if (n + 1) * theta > math.pi else 0),
                                     rel=1e-9, abs=1e-12)
        assert np.linalg.norm(r.p[0]) == pytest.approx(p0, rel=1e-13)
    xs = np.array(xs)
    v = p0 / (g * K.ME)
    Rad = v * r.dt / 2 / math.sin(theta / 2)
    # circumcentre of three successive positions
    a, b, c = xs[0], xs[4], xs[8]
    d = 2 * (a[0] * (b[1] - c[1]) + b[0] * (c[1] - a[1]) + c[0] * (a[1] - b[1]))
    ux = ((a @ a) * (b[1] - c[1]) + (b @ b) * (c[1] - a[1]) + (c @ c) * (a[1] - b[1])) / d
    uy = ((a @ a) * (c[0] - b[0]) + (b @ b) * (a[0] - c[0]) + (c @ c) * (b[0] - a[0])) / d
    radii = np.hypot(xs[:, 0] - ux, xs[:, 1] - uy)
    assert np.allclose(radii, Rad, rtol=1e-9)


def test_uniform_electric_field_closed_form():
    """Uniform E, B = 0: p(t) = p0 + q E t exactly."""
    Ex = 3e9
    p0 = PT.momentum_of_energy(2.0 * MEV)
    r = _one_particle_run([10.2e-6, 16e-6, 16e-6], [p0, 0.0, 0.0], R.PHYS_FIELDS)
    shape = r.E[0].shape
    r.E = (np.full(shape, Ex), np.zeros(shape), np.zeros(shape))
    for n in range(5):
        r.step()
    assert r.p[0, 0] == pytest.approx(p0 - K.E * Ex * 5 * r.dt, rel=1e-13)
    # the ledger records the work as field loss
    eps_end = PT.kinetic(r.p)[0]
    assert r.ledger["field_loss"] == pytest.approx(PT.kinetic(np.array([[p0, 0, 0]]))[0] - eps_end, rel=1e-10)


def _icru37_collision_stopping(eps, Z, n_i, I):
    """Electron collision stopping power of ICRU Report 37 (Rohrlich-Carlson
    form of the Bethe formula), density effect omitted, written out
    independently of the paper's eq. (stop_ion)."""
    tau = eps / K.MEC2
    g = tau + 1
    b2 = 1 - 1 / g ** 2
    Fm = 1 - b2 + (tau ** 2 / 8 - (2 * tau + 1) * math.log(2)) / (tau + 1) ** 2
    return (2 * math.pi * K.R_E ** 2 * K.MEC2 * Z * n_i / b2
            * (math.log(tau ** 2 * (tau + 2) / (2 * (I / K.MEC2) ** 2)) + Fm))


@pytest.mark.parametrize("mat", ["Al", "Au"])
@pytest.mark.parametrize("eps_mev", [0.03, 0.3, 1.0, 10.0, 100.0])
def test_stop_ion_agrees_with_bethe_icru37(mat, eps_mev):
    m = W.MATERIALS[mat]
    n_i = m["rho"] / (m["A"] * K.AMU)
    I = 11 * K.E * m["Z"]
    eps = eps_mev * MEV
    p = np.array([[PT.momentum_of_energy(eps), 0, 0]])
    S = PT.stopping_ion(np.array([eps]), p, m["Z"], n_i, I)[0]
    assert S == pytest.approx(_icru37_collision_stopping(eps, m["Z"], n_i, I), rel=0.02)


def test_ionisation_step_loss():
    """One step with only ionisation: Delta eps = S(eps) v dt (well below eps)."""
    p0 = PT.momentum_of_energy(1.5 * MEV)
    r = _one_particle_run([10.5e-6, 16e-6, 16e-6], [0.0, p0, 0.0], R.PHYS_ION)
    eps0 = PT.kinetic(r.p)[0]
    g = math.sqrt(1 + (p0 / (K.ME * K.C)) ** 2)
    v = p0 / (g * K.ME)
    m = W.MATERIALS["Au"]
    n_i = m["rho"] / (m["A"] * K.AMU)
    S = _icru37_collision_stopping(eps0, 79.0, n_i, 11 * K.E * 79)
    r.step()
    dE = eps0 - PT.kinetic(r.p)[0]
    assert dE == pytest.approx(S * v * r.dt, rel=0.02)
    assert r.ledger["ionisation"] == pytest.approx(dE, rel=1e-10)
    assert np.sum(r.ion_heat) == pytest.approx(dE, rel=1e-10)


def test_davies_variance_is_classical_multiple_scattering():
    """Davies' variance per unit path equals the classical small-angle multiple
    scattering rate 8 pi n Z^2 r_e^2 (m c^2/(p v))^2 ln(Lambda), with the
    logarithm's argument 2 a_B Z^-1/3 p / hbar (screening radius over the
    reduced de Broglie length)."""
    Z, n_i, dt = 79.0, 5.9e28, 1e-14
    for eps_mev in (0.2, 1.0, 20.0):
        pm = PT.momentum_of_energy(eps_mev * MEV)
        g = math.sqrt(1 + (pm / (K.ME * K.C)) ** 2)
        v = pm / (g * K.ME)
        lnL = math.log(2 * K.A_BOHR * Z ** (-1 / 3) * pm / K.HBAR)
        rossi = 8 * math.pi * n_i * Z ** 2 * K.R_E ** 2 * (K.MEC2 / (pm * v)) ** 2 * lnL * v * dt
        s2 = PT.davies_sigma2(np.array([[0, pm, 0]]), Z, n_i, dt)[0]
        assert s2 == pytest.approx(rossi, rel=1e-8)   # h vs 2 pi hbar rounding in CODATA


def test_davies_scatter_statistics():
    """Over many particles, the deflection angle of one step has the mean square
    of the Davies formula (Box-Muller normal, rotation keeps |p|)."""
    n = 40000
    pm = PT.momentum_of_energy(5.0 * MEV)
    rng = np.random.default_rng(3)
    pos = np.column_stack([rng.uniform(2e-6, 30e-6, n), rng.uniform(2e-6, 30e-6, n),
                           rng.uniform(2e-6, 30e-6, n)])
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = _one_particle_run(pos, d * pm, R.PHYS_SCATTER, dt=1e-15)
    r.box_lo[:] = -1e12
    r.box_hi[:] = 1e12
    p_before = r.p.copy()
    r.step()
    cosang = np.sum(p_before * r.p, axis=1) / (pm * np.linalg.norm(r.p, axis=1))
    ang = np.arccos(np.clip(cosang, -1, 1))
    s2 = PT.davies_sigma2(p_before[:1], 79.0, r.n_i, r.dt)[0]
    assert np.allclose(np.linalg.norm(r.p, axis=1), pm, rtol=1e-13)
    assert np.mean(ang ** 2) == pytest.approx(s2, rel=0.03)


def test_photon_polar_angle_distribution():
    """gamma theta follows the Tsai-based mixture 1/4 Gamma(2, a) + 3/4
    Gamma(2, 3a), a = 0.625: Kolmogorov-Smirnov against the closed-form CDF
    1 - exp(-k u)(1 + k u) of each component, and the mean 2/a (1/4 + 1/4)."""
    gam = 40.0
    n = 100000
    rng = np.random.default_rng(5)
    th = PT.photon_polar(np.full(n, gam), rng.random(n), rng.random(n))
    u = th * gam
    a = 0.625
    G = lambda x, k: 1.0 - np.exp(-k * x) * (1.0 + k * x)
    assert stats.kstest(u, lambda x: 0.25 * G(x, a) + 0.75 * G(x, 3 * a)).pvalue > 1e-3
    assert np.mean(u) == pytest.approx(1.6, rel=0.01)
    # the cap at pi for slow electrons
    assert PT.photon_polar(np.array([1.0]), np.array([0.9]), np.array([1e-6]))[0] == pytest.approx(math.pi)


def test_optical_depth_emission_probability():
    """Fresh tau_e ~ Exp(1): the chance of an emission within one step is
    exactly 1 - exp(-dtau)."""
    cfg = W.base_config(nx=32, ny=32, nz=32, x_lo=0.0, x_hi=32e-6, physics=R.PHYS_BREM,
                        brem_boost=10.0, max_particles=1, series_len=4)
    r = OracleRun(cfg)
    n = 60000
    eps = 20 * MEV
    rng = np.random.default_rng(9)
    pos = np.column_stack([rng.uniform(1e-6, 31e-6, n) for _ in range(3)])
    from oracle import philox as P
    ids = np.arange(n, dtype=np.uint32)
    tau = -np.log(1 - P.uniforms(ids, 123, 0, 5)[0])
    r.set_state(dict(pos=pos, p=np.tile([0, 0, PT.momentum_of_energy(eps)], (n, 1)),
                     w=np.ones(n), tau=tau, ids=ids))
    g = 1 + eps / K.MEC2
    beta = math.sqrt(1 - 1 / g ** 2)
    dtau = 10.0 * r.n_i * r.cz * float(r.table.sigma(eps)) * beta * K.C * r.dt
    r.step()
    frac = r.counters["n_emitted"] / n
    expect = 1 - math.exp(-dtau)
    assert frac == pytest.approx(expect, abs=4 * math.sqrt(expect * (1 - expect) / n))
    # energy bookkeeping of the emissions: photon energy = electron loss
    assert r.ledger["rad_discrete"] == pytest.approx(
        float(np.sum(r.hist_E) + r.flow[0] + r.flow[2]), rel=1e-12)


def test_reflux_paper_mode_single_event():
    """An electron crossing x_hi is mirrored, loses kappa_tnsa a0 m c of |p|,
    is turned by (u - 1/2) sigma and sent back inward (Sec. II.A)."""
    cfg_over = dict(I0=1e26)
    p0 = PT.momentum_of_energy(3.0 * MEV)
    r = _one_particle_run([31.9e-6, 16e-6, 16e-6], [p0, 0.0, 0.0], 0, **cfg_over)
    r.step()
    a0 = PT.a0_of(1e26, 1e-6)
    assert np.linalg.norm(r.p[0]) == pytest.approx(p0 - 2.7e-3 * a0 * K.ME * K.C, rel=1e-12)
    assert r.p[0, 0] < 0
    g = math.sqrt(1 + (p0 / (K.ME * K.C)) ** 2)
    x_expect = 2 * 32e-6 - (31.9e-6 + p0 / (g * K.ME) * r.dt)
    assert r.pos[0, 0] == pytest.approx(x_expect, rel=1e-12)
    from oracle import philox as P
    u = P.uniforms(np.array([0]), 0, 0, P.SLOT_REFLUX[0])
    dth = abs((u[0][0] - 0.5) * math.radians(23))
    ang = math.acos(-r.p[0, 0] / np.linalg.norm(r.p[0]))
    assert ang == pytest.approx(dth, rel=1e-9)
    eps_after = PT.kinetic(r.p)[0]
    eps0 = PT.kinetic(np.array([[p0, 0, 0]]))[0]
    assert r.ledger["reflux"] == pytest.approx(eps0 - eps_after, rel=1e-9)
    assert r.counters["n_reflux"] == 1


def test_reflux_energy_fraction_mode_and_escape():
    p_lo = PT.momentum_of_energy(3.0 * MEV)
    r = _one_particle_run([31.9e-6, 16e-6, 16e-6], [p_lo, 0.0, 0.0], 0, reflux_ke_frac=0.01)
    eps0 = PT.kinetic(r.p)[0]
    r.step()
    assert PT.kinetic(r.p)[0] == pytest.approx(0.99 * eps0, rel=1e-12)
    # above kappa_esc a0 m c^2 the electron escapes and its energy is booked
    a0 = PT.a0_of(1e24, 1e-6)
    eps_hi = 2.0 * a0 * K.MEC2 * 1.01
    r = _one_particle_run([31.9e-6, 16e-6, 16e-6], [PT.momentum_of_energy(eps_hi), 0, 0], 0)
    r.step()
    assert r.alive.sum() == 0
    assert r.ledger["escaped"] == pytest.approx(eps_hi, rel=1e-12)


def test_low_energy_removal_heats_cell():
    p0 = PT.momentum_of_energy(5e3 * K.E)
    r = _one_particle_run([10.5e-6, 12.5e-6, 3.5e-6], [p0, 0, 0], 0)
    r.step()
    assert r.alive.sum() == 0
    eps0 = 5e3 * K.E
    assert r.ledger["stopped"] == pytest.approx(eps0, rel=1e-12)
    assert r.ion_heat[10, 12, 3] == pytest.approx(eps0, rel=1e-12)


# --------------------------------------------------------------------------
# injection
# --------------------------------------------------------------------------
def test_injection_samplers():
    src = W.source(n_macro=200000, r_fwhm=5e-6, T_hot=2.0 * MEV, half_angle=math.radians(30))
    X, p, w, tau, ids = PT.inject(src, 0, 200000, 0, 11, 2, 1e-6, 1e24)
    pos = X * 1e-6
    eps = PT.kinetic(p)
    assert np.mean(eps) == pytest.approx(2.0 * MEV, rel=0.01)
    r = np.hypot(pos[:, 1] - src["y0"], pos[:, 2] - src["z0"])
    assert r.max() <= 2.5e-6 * (1 + 1e-12)
    # electrons are placed with areal density proportional to f, so the
    # sample mean of 1/f is the disc area over int f dA = 1/<f> = 2 ln 2
    f = 2.0 ** (-(2 * r / 5e-6) ** 2)
    assert np.mean(1.0 / f) == pytest.approx(2 * math.log(2), rel=0.003)
    cdf_r2 = lambda s: 2 * (1 - 2.0 ** (-4 * s / 25e-12))   # P(r^2 <= s), f >= 1/2 disc
    assert stats.kstest(r ** 2, cdf_r2).pvalue > 1e-3
    ct = p[:, 0] / np.linalg.norm(p, axis=1)
    cm = math.cos(math.radians(30))
    assert stats.kstest((1 - ct) / (1 - cm), "uniform").pvalue > 1e-3
    assert stats.kstest(tau, "expon").pvalue > 1e-3
    assert np.all(X[:, 0] == 2.0)


def test_injection_schedule_counts():
    src = W.source(n_macro=1003, t_start=0.0, t_end=1e-12)
    s0, ns = PT.injection_schedule(src, 1e-14)
    assert (s0, ns) == (0, 100)
    cfg = W.base_config(max_particles=2048, series_len=4)
    r = OracleRun(cfg)
    r.add_source(src)
    counts = []
    for n in range(101):
        before = len(r.ids)
        r._inject(n)
        counts.append(len(r.ids) - before)
    assert sum(counts) == 1003 and counts[:3] == [11, 11, 11] and counts[3] == 10 and counts[100] == 0
    assert np.array_equal(r.ids, np.arange(1003))


def test_printed_envelope_means(golden_dir):
    """<fg> ~ 0.41 and <sqrt(fg)> ~ 0.61 (Sec. II.B) with f = 2^-(2r/r_fwhm)^2
    averaged over the disc f >= 1/2 and g = 2^-(2t/t_fwhm)^2 over g >= 1/10 --
    the envelope reading that also fixes the spot sampler's truncation."""
    nums = json.load(open(os.path.join(golden_dir, "paper_numbers.json")))
    R_ = 0.5
    fmean = integrate.quad(lambda r: 2 ** (-(2 * r) ** 2) * 2 * r, 0, R_)[0] / R_ ** 2
    sfmean = integrate.quad(lambda r: 2 ** (-(2 * r) ** 2 / 2) * 2 * r, 0, R_)[0] / R_ ** 2
    tm = 0.5 * math.sqrt(math.log(10) / math.log(2))
    gmean = integrate.quad(lambda t: 2 ** (-(2 * t) ** 2), 0, tm)[0] / tm
    sgmean = integrate.quad(lambda t: 2 ** (-(2 * t) ** 2 / 2), 0, tm)[0] / tm
    assert fmean == pytest.approx(1 / (2 * math.log(2)), rel=1e-10)
    assert round(fmean * gmean, 2) == nums["mean_fg"]["value"]
    assert round(sfmean * sgmean, 2) == nums["mean_sqrt_fg"]["value"]


def test_default_weight_conserves_energy():
    src = W.source(n_macro=5000, r_fwhm=5e-6, T_hot=1.0 * MEV, t_end=1e-12, eta_l2e=0.3)
    w = PT.default_weight(src, 1e24)
    energy = 1e24 * (1 / (2 * math.log(2))) * math.pi * (5e-6) ** 2 / 4 * 1e-12 * 0.3
    assert w * 5000 * 1.0 * MEV == pytest.approx(energy, rel=1e-12)
