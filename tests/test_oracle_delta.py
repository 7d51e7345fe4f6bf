"""Oracle pins for delta rays and the restricted ionisation loss (App. B):
the restricted stopping power against the unrestricted Bethe formula for
electrons, the split of the loss at the cut against the Moller
cross-section, the cross-section's symmetry and non-relativistic limit, the
density effect's plateau, the energy sampler against the cross-section, the
two-body kinematics, and one step's emission rate, ledger and ids."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W
from oracle import OracleRun
from oracle import constants as K
from oracle import moller as M
from oracle import particles as PT
from oracle import run as R
from oracle import solid as S

MEV = 1e6 * K.E
KEV = 1e3 * K.E
AU = W.MATERIALS["Au"]
N_I = S.ion_density(AU["rho"], AU["A"])
Z = AU["Z"]
I_EX = 11.0 * K.E * Z


def _bethe_unrestricted(eps, I_ex):
    """ICRU-37 electron stopping power without density effect, with the
    Rohrlich-Carlson F^-(t) = 1 - beta^2 + (t^2/8 - (2t + 1) ln 2)/(t + 1)^2:
    2 pi r_e^2 m c^2 Z n_i / beta^2 (ln(t^2 (t + 2) / (2 (I/mc^2)^2)) + F^-)."""
    t = eps / K.MEC2
    b2 = 1.0 - 1.0 / (t + 1.0) ** 2
    F = 1.0 - b2 + (t * t / 8.0 - (2.0 * t + 1.0) * math.log(2.0)) / (t + 1.0) ** 2
    return (2.0 * math.pi * K.R_E ** 2 * K.MEC2 * Z * N_I / b2
            * (math.log(t * t * (t + 2.0) / (2.0 * (I_ex / K.MEC2) ** 2)) + F))


def test_no_cut_below_the_energy_is_the_unrestricted_bethe_formula():
    """With the cut above eps/2 no delta ray is possible (the faster electron
    is the primary) and the restricted form is the whole Bethe loss; at
    these energies gold's density effect (high-energy form) is zero."""
    for e in (0.05, 0.3, 1.0, 3.0):
        eps = e * MEV
        assert float(M.density_effect(math.sqrt((eps / K.MEC2 + 1) ** 2 - 1), Z, N_I, I_EX)) == 0.0
        got = float(M.restricted_stopping(np.array([eps]), Z, N_I, I_EX, 1e3 * MEV)[0])
        assert got == pytest.approx(_bethe_unrestricted(eps, I_EX), rel=1e-12)


@pytest.mark.parametrize("e_mev", [0.05, 0.5, 2.0, 20.0, 200.0])
def test_loss_split_at_the_cut_matches_the_moller_cross_section(e_mev):
    """restricted(cut) + n_i * integral of eps_d dsigma over [cut, eps/2]
    = restricted(no cut): F^- and d sigma/dx describe the same collisions."""
    eps = e_mev * MEV
    cut = 1 * KEV
    lo = float(M.restricted_stopping(np.array([eps]), Z, N_I, I_EX, cut)[0])
    full = float(M.restricted_stopping(np.array([eps]), Z, N_I, I_EX, eps)[0])
    xc = cut / eps
    integral, err = integrate.quad(lambda x: x * float(M.moller_dxs(x, eps, Z)),
                                   xc, 0.5, limit=400, epsabs=0.0, epsrel=1e-12,
                                   points=[min(0.5, 10 * xc), min(0.5, 100 * xc)])
    assert lo + N_I * eps * integral == pytest.approx(full, rel=1e-9)


@pytest.mark.parametrize("e_mev", [0.01, 0.3, 5.0, 100.0])
def test_total_cross_section_is_the_integral(e_mev):
    eps = e_mev * MEV
    cut = 1 * KEV
    xc = cut / eps
    q, _ = integrate.quad(lambda x: float(M.moller_dxs(x, eps, Z)), xc, 0.5, limit=400,
                          epsabs=0.0, epsrel=1e-12, points=[min(0.5, 10 * xc)])
    assert float(M.moller_sigma(np.array([eps]), Z, cut)[0]) == pytest.approx(q, rel=1e-10)
    # nothing above the cut once eps <= 2 cut
    assert float(M.moller_sigma(np.array([1.9 * cut]), Z, cut)[0]) == 0.0


def test_moller_symmetry_and_nonrelativistic_limit():
    """Two identical electrons: d sigma/dx(x) = d sigma/dx(1 - x).  As
    gamma -> 1 the bracket becomes Mott's 1/x^2 + 1/(1-x)^2 - 1/(x(1-x))."""
    x = np.linspace(0.01, 0.99, 57)
    for e in (1 * KEV, 1 * MEV, 50 * MEV):
        assert np.allclose(M.moller_dxs(x, e, Z), M.moller_dxs(1 - x, e, Z), rtol=1e-12)
    eps = 1e-3 * K.E        # 1 meV: gamma - 1 ~ 2e-9
    g = 1 + eps / K.MEC2
    b2 = 1 - 1 / g ** 2
    mott = 1 / x ** 2 + 1 / (1 - x) ** 2 - 1 / (x * (1 - x))
    br = M.moller_dxs(x, eps, Z) * b2 * (g - 1) / (2 * math.pi * K.R_E ** 2 * Z)
    assert np.allclose(br, mott, rtol=1e-7)


def test_density_effect_gives_the_fermi_plateau():
    """At high energy the density effect cancels the excitation energy: the
    restricted loss no longer depends on I."""
    eps = np.array([5e3 * MEV, 5e4 * MEV])
    a = M.restricted_stopping(eps, Z, N_I, I_EX, 1 * KEV)
    b = M.restricted_stopping(eps, Z, N_I, 2.0 * I_EX, 1 * KEV)
    assert np.allclose(a, b, rtol=1e-12)
    # and it is active there: without it the loss would grow
    assert np.all(M.density_effect(eps / K.MEC2, Z, N_I, I_EX) > 5.0)


@pytest.mark.parametrize("e_mev", [0.02, 0.5, 5.0, 200.0])
def test_sampler_draws_the_moller_spectrum(e_mev):
    """Energies from the rejection sampler follow d sigma/dx on [x_c, 1/2]
    (Kolmogorov-Smirnov against the cross-section's own CDF)."""
    eps = e_mev * MEV
    cut = 1 * KEV
    n = 20000
    rng = np.random.default_rng(11)
    u = rng.random((M.N_TRIES, 2, n))
    x = M.sample_fraction(np.full(n, eps), cut, u)
    xc = cut / eps
    assert np.all((x >= xc) & (x <= 0.5))
    tot = float(M.moller_sigma(np.array([eps]), Z, cut)[0])

    def cdf(v):
        return np.array([integrate.quad(lambda s: float(M.moller_dxs(s, eps, Z)), xc, t,
                                        limit=200, points=[min(t, 10 * xc)])[0] for t in np.atleast_1d(v)]) / tot

    grid = np.quantile(x, np.linspace(0, 1, 41)[1:-1])
    emp = np.searchsorted(np.sort(x), grid, side="right") / n
    assert np.max(np.abs(emp - cdf(grid))) < 1.63 / math.sqrt(n) * 1.5


def test_two_body_kinematics_conserve_energy_and_momentum():
    """The delta ray's polar angle is the one for which p - p_d has exactly
    the momentum of eps - eps_d; non-relativistically the two electrons
    leave at right angles."""
    rng = np.random.default_rng(3)
    n = 200
    eps = rng.uniform(0.01, 50, n) * MEV
    d = rng.normal(size=(n, 3))
    p = d / np.linalg.norm(d, axis=1)[:, None] * PT.momentum_of_energy(eps)[:, None]
    e_d = eps * rng.uniform(1e-4, 0.5, n)
    q, dd = M.delta_kinematics(p, eps, e_d, rng.uniform(0, 2 * np.pi, n))
    raw = p - dd
    assert np.allclose(np.linalg.norm(raw, axis=1), PT.momentum_of_energy(eps - e_d), rtol=1e-9)
    assert np.allclose(PT.kinetic(dd), e_d, rtol=1e-12)
    assert np.allclose(q, raw, rtol=1e-8, atol=1e-9 * np.linalg.norm(p, axis=1).max())
    # non-relativistic: opening angle 90 deg
    e0 = np.full(4, 1e-2 * K.E)
    p0 = np.array([[1.0, 0, 0]] * 4) * PT.momentum_of_energy(e0)[:, None]
    q0, d0 = M.delta_kinematics(p0, e0, e0 * np.array([0.1, 0.2, 0.3, 0.45]), np.zeros(4))
    cosang = np.sum(q0 * d0, axis=1) / (np.linalg.norm(q0, axis=1) * np.linalg.norm(d0, axis=1))
    assert np.allclose(cosang, 0.0, atol=1e-6)


def _delta_run(n, eps, phys=R.PHYS_ION | R.PHYS_DELTA, pos=None, dt=10e-15, taud=None):
    cfg = W.base_config(nx=16, ny=16, nz=16, x_lo=0.0, x_hi=16e-6, dt=dt, physics=phys,
                        max_particles=1 << 20, series_len=4)
    r = OracleRun(cfg)
    if pos is None:
        pos = np.tile([[6.3e-6, 7.1e-6, 8.6e-6]], (n, 1))
    p = np.column_stack([PT.momentum_of_energy(eps), np.zeros(n), np.zeros(n)])
    rng = np.random.default_rng(5)
    taud = rng.exponential(size=n) if taud is None else taud
    r.set_state(dict(pos=pos, p=p, w=np.full(n, 2.0), tau=np.full(n, 30.0), tau_d=taud,
                     ids=np.arange(n, dtype=np.uint32)))
    return r


def test_one_step_emission_rate_energy_and_ledger():
    """20000 electrons of 2 MeV with exponential depths: the fraction that
    emits is 1 - exp(-n_i sigma v dt), each emitter gives its delta ray the
    sampled energy, the ledger closes, and the delta rays are born at x^n
    with the parent's weight."""
    n = 20000
    eps = np.full(n, 2.0 * MEV)
    r = _delta_run(n, eps)
    e1 = r.kinetic_total()
    r.step()
    t = eps[0] / K.MEC2
    b = math.sqrt(1 - 1 / (t + 1) ** 2)
    # the restricted loss comes first; the delta-ray depth uses the energy after it
    S_r = float(M.restricted_stopping(eps[:1], Z, N_I, I_EX, 1 * KEV)[0])
    e2 = eps[0] - S_r * b * K.C * r.dt
    b2 = math.sqrt(1 - 1 / (e2 / K.MEC2 + 1) ** 2)
    dtau = N_I * float(M.moller_sigma(np.array([e2]), Z, 1 * KEV)[0]) * b2 * K.C * r.dt
    pe = 1 - math.exp(-dtau)
    k = r.counters["n_delta"]
    assert abs(k - n * pe) < 5 * math.sqrt(n * pe * (1 - pe))
    L = r.ledger
    assert abs(e1 - (r.kinetic_total() + L["ionisation"] + L["stopped"] + L["residual"])) < 1e-12 * e1
    new = r.ids >= R.DELTA_ID_BIT
    born = int(np.sum(new))
    assert born + r.counters["n_delta_lost"] <= k
    assert np.allclose(r.X[new] * r.dx, [6.3e-6, 7.1e-6, 8.6e-6], rtol=0, atol=1e-18)
    assert np.all(r.w[new] == 2.0)
    # energy taken from the parents equals the delta rays' plus the stopped ones'
    ekin_new = float(np.sum(r.w[new] * PT.kinetic(r.p[new])))
    assert ekin_new + r.ledger["stopped"] == pytest.approx(
        e1 - r.ledger["ionisation"] - float(np.sum(r.w[~new] * PT.kinetic(r.p[~new]))), rel=1e-9)
    # the mean delta-ray energy is the cross-section's (5 sigma of the sample mean)
    xc = 1 * KEV / e2
    tot = float(M.moller_sigma(np.array([e2]), Z, 1 * KEV)[0])
    m1, m2 = (integrate.quad(lambda s, q=q: s ** q * float(M.moller_dxs(s, e2, Z)), xc, 0.5,
                             limit=400, points=[10 * xc])[0] / tot for q in (1, 2))
    e_given = e1 - r.ledger["ionisation"] - float(np.sum(r.w[~new] * PT.kinetic(r.p[~new])))
    mean = e_given / 2.0 / k / e2        # weights are 2
    assert abs(mean - m1) < 5 * math.sqrt((m2 - m1 * m1) / k)


def test_delta_ray_ids_follow_tile_then_parent_order():
    """Parents in two tiles: the delta rays of the lower tile come first, each
    tile's in parent-id order; a second step continues the numbering."""
    n = 4000
    eps = np.full(n, 5.0 * MEV)
    pos = np.zeros((n, 3))
    pos[:, 1:] = 5.5e-6
    # even ids in tile x = 2 (cells 8..11), odd ids in tile x = 0
    pos[:, 0] = np.where(np.arange(n) % 2 == 0, 9.5e-6, 1.5e-6)
    r = _delta_run(n, eps, pos=pos, dt=20e-15)
    st0 = r.state()
    r.step()
    new = r.ids >= R.DELTA_ID_BIT
    ids = r.ids[new]
    assert np.array_equal(ids, R.DELTA_ID_BIT + np.arange(len(ids)))
    x = r.X[new, 0]
    tile0 = x < 4
    assert tile0.any() and (~tile0).any()
    # all tile-0 rays (x ~ 1.5 cells) before the tile-2 ones
    assert np.all(np.diff(tile0.astype(int)) <= 0)
    first = int(len(ids))
    r.step()
    ids2 = np.sort(r.ids[r.ids >= R.DELTA_ID_BIT + first])
    assert len(ids2) > 0
    assert np.array_equal(ids2, R.DELTA_ID_BIT + first + np.arange(len(ids2)))
    assert r.delta_next == first + len(ids2)
    assert st0["delta_next"] == 0
