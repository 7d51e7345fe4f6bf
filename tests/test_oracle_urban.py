"""Oracle pins for the Urban-type elastic scatter (App. B): the transport
cross-sections against quadrature of the screened Rutherford law written
here in SI, the model function's Legendre moments against the Lewis values,
the sampler against its CDF, the small-step limit against the Davies
variance, and isotropy for long steps."""
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
from oracle import urban as U

MEV = 1e6 * K.E
TA = W.MATERIALS["Ta"]
AU = W.MATERIALS["Au"]


def _elem(mat):
    return S.element(mat["Z"], mat["A"], mat["rho"])


def _rutherford_screened(mu, eps, Z):
    """d sigma / d Omega [m^2/sr] of Z(Z+1) point charges seen by an
    electron of kinetic energy eps, screened by Moliere's angle: written
    from p, v in SI and the Thomas-Fermi radius 0.885 a_0 Z^-1/3."""
    g = 1.0 + eps / (K.ME * K.C ** 2)
    p = K.ME * K.C * math.sqrt(g * g - 1.0)
    v = p / (g * K.ME)
    chi0 = K.HBAR / (p * 0.88534 * K.A_BOHR * Z ** (-1.0 / 3.0))
    A = chi0 ** 2 / 4.0 * (1.13 + 3.76 * (Z * K.E ** 2 / (4 * math.pi * K.EPS0 * K.HBAR * v)) ** 2)
    pre = Z * (Z + 1.0) * (K.E ** 2 / (4.0 * math.pi * K.EPS0)) ** 2 / (4.0 * (p * v) ** 2)
    return pre / (mu + A) ** 2, A


@pytest.mark.parametrize("Z", [6.0, 29.0, 73.0])
@pytest.mark.parametrize("e_mev", [0.02, 0.5, 5.0])
def test_transport_cross_sections_match_quadrature(Z, e_mev):
    """sigma_l = int (1 - P_l(cos chi)) d sigma over the sphere, computed by
    quadrature in ln mu (d Omega = 4 pi d mu, mu = (1 - cos chi)/2)."""
    eps = e_mev * MEV
    _, A = _rutherford_screened(0.0, eps, Z)
    s1, s2 = U.transport_xs(np.array([eps]), Z)

    def integral(weight):
        f = lambda t: (4.0 * math.pi * _rutherford_screened(math.exp(t), eps, Z)[0]
                       * weight(math.exp(t)) * math.exp(t))
        lo = math.log(A) - 30.0
        pts = [math.log(A) + k for k in (-5.0, 0.0, 5.0) if math.log(A) + k < 0.0]
        return integrate.quad(f, lo, 0.0, points=pts, limit=400, epsrel=1e-12)[0]

    q1 = integral(lambda m: 2.0 * m)                      # 1 - cos chi
    q2 = integral(lambda m: 6.0 * m * (1.0 - m))          # 1 - P_2(cos chi)
    assert s1[0] == pytest.approx(q1, rel=1e-8)
    assert s2[0] == pytest.approx(q2, rel=1e-8)
    # Moliere's A, the same in the oracle's units
    um = PT.momentum_of_energy(eps) / (K.ME * K.C)
    beta = um / math.sqrt(1 + um * um)
    assert U.screening(um, beta, Z) == pytest.approx(A, rel=1e-12)


def _cases():
    """(x_1, x_2) of real steps: Ta at 5 fs and Au at 20 fs, 10 keV-50 MeV."""
    out = []
    for mat, dt in ((TA, 5e-15), (AU, 20e-15), (W.MATERIALS["Al"], 20e-15)):
        eps = np.logspace(-2, np.log10(50.0), 25) * MEV
        x1, x2 = U.lewis_x(eps, [_elem(mat)], dt)
        out += list(zip(x1, x2))
    return np.array(out)


def _legendre_moments(a, wi):
    """1 - <P_1> and 1 - <P_2> of the model density by quadrature in
    w = 1 - u (1 - P_1 = w, 1 - P_2 = 3 w (2 - w) / 2)."""
    f = lambda w, l: U.model_density(1.0 - w, a, wi) * (w if l == 1 else 1.5 * w * (2.0 - w))
    cut = min(2.0, 60.0 / a)
    res = []
    for l in (1, 2):
        v = integrate.quad(f, 0.0, cut, args=(l,), points=[min(cut, 1.0 / a)], limit=400, epsrel=1e-13)[0]
        if cut < 2.0:
            v += integrate.quad(f, cut, 2.0, args=(l,), limit=400, epsrel=1e-13)[0]
        res.append(v)
    return res


def test_model_function_has_the_lewis_moments():
    """Where w_i >= 0 the mixture's first two Legendre moments are exp(-x_1)
    and exp(-x_2) (Lewis), by quadrature of its density; where the match
    would need w_i < 0, w_i = 0 and the first moment still holds."""
    c = _cases()
    a, wi = U.model_params(c[:, 0], c[:, 1])
    assert np.all(wi >= 0.0) and np.all(wi <= 1.0) and np.all(a > 0.0)
    n_full = 0
    for (x1, x2), ai, wii in zip(c, a, wi):
        m1, m2 = _legendre_moments(ai, wii)
        assert m1 == pytest.approx(-math.expm1(-x1), rel=1e-9)
        if wii > 0.0:
            n_full += 1
            assert m2 == pytest.approx(-math.expm1(-x2), rel=1e-9)
    assert n_full > 0.9 * len(c)


def test_fallback_case():
    """Au at 100 keV over 20 fs is one of the long steps where both moments
    cannot be matched with w_i >= 0: the first is."""
    x1, x2 = U.lewis_x(np.array([0.1 * MEV]), [_elem(AU)], 20e-15)
    a, wi = U.model_params(x1, x2)
    assert wi[0] == 0.0
    assert U.langevin(a)[0] == pytest.approx(math.exp(-x1[0]), rel=1e-12)


def test_langevin_against_high_precision():
    """coth a - 1/a, and 1/L - 3/a where the series serves, against
    40-digit arithmetic on both sides of the switch and far out."""
    import mpmath as mp
    mp.mp.dps = 40
    a = np.array([1e-6, 0.01, 0.3, 0.5, 0.9, 0.989128, 0.999999, 1.0, 1.2, 3.0, 30.0, 1e6])
    ref = np.array([float(mp.coth(mp.mpf(x)) - 1 / mp.mpf(x)) for x in a])
    assert np.allclose(U.langevin(a), ref, rtol=3e-16, atol=0)
    small = a[a < 1.0]
    ref_phi = np.array([float(1 / (mp.coth(mp.mpf(x)) - 1 / mp.mpf(x)) - 3 / mp.mpf(x)) for x in small])
    assert np.allclose(U._phi_small(small), ref_phi, rtol=1e-15, atol=0)
    assert U.langevin(np.array([1e6]))[0] == pytest.approx(1 - 1e-6, rel=1e-15)


def test_model_parameters_against_high_precision():
    """The solved (a, w_i) of a few real steps against the same equations
    solved in 40-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 40
    c = _cases()[::7]
    a, wi = U.model_params(c[:, 0], c[:, 1])
    for (x1, x2), ai, wii in zip(c, a, wi):
        L = lambda t: mp.coth(t) - 1 / t
        if wii > 0.0:
            am = mp.findroot(lambda t: 1 / L(t) - 3 / t - mp.exp(mp.mpf(x1) - mp.mpf(x2)), mp.mpf(ai))
            assert float(1 - mp.exp(-mp.mpf(x1)) / L(am)) == pytest.approx(wii, rel=1e-11, abs=1e-15)
        else:
            am = mp.findroot(lambda t: L(t) - mp.exp(-mp.mpf(x1)), mp.mpf(ai))
        assert ai == pytest.approx(float(am), rel=3e-14)


def test_sampler_moments_and_cdf():
    """4e5 draws: the sample means of 1 - P_1 and 1 - P_2 within 5 standard
    errors of the Lewis values, and the core's draws follow its CDF."""
    rng = np.random.default_rng(11)
    for x1, x2 in ((0.02, 0.053), (0.4, 0.95)):
        a, wi = U.model_params(np.array([x1]), np.array([x2]))
        n = 400_000
        ua, ub = rng.random(n), 1.0 - rng.random(n)     # ub in (0, 1]
        w = U.one_minus_cos(a[0], wi[0], ua, ub)
        assert np.all((w >= 0.0) & (w <= 2.0))
        for l, val in ((1, w), (2, 1.5 * w * (2.0 - w))):
            target = -math.expm1(-(x1 if l == 1 else x2))
            assert abs(val.mean() - target) < 5.0 * val.std() / math.sqrt(n)
        core = w[ua >= wi[0]]
        cdf = lambda x: -np.expm1(-a[0] * x) / -math.expm1(-2.0 * a[0])
        assert stats.kstest(core, cdf).pvalue > 1e-3


def test_small_steps_approach_the_davies_variance():
    """For short steps the polar variance 2 (1 - <cos theta>) is 2 s /
    lambda_1, the same physics as the Davies variance (App. B) up to the
    screening logarithm: within 30 % for MeV electrons in gold and
    tantalum."""
    for mat in (AU, TA):
        eps = np.array([1.0, 3.0, 10.0]) * MEV
        dt = 1e-16
        x1, _ = U.lewis_x(eps, [_elem(mat)], dt)
        p = np.zeros((3, 3))
        p[:, 0] = PT.momentum_of_energy(eps)
        dav = PT.davies_sigma2(p, mat["Z"], S.ion_density(mat["rho"], mat["A"]), dt)
        ratio = 2.0 * x1 / dav
        print(f"  Z={mat['Z']:.0f}: Urban-type / Davies variance {np.round(ratio, 3)}")
        assert np.all((ratio > 0.7) & (ratio < 1.3))


def test_long_steps_are_isotropic():
    """x_1 large: every moment vanishes and the density is flat."""
    a, wi = U.model_params(np.array([60.0, 40.0]), np.array([70.0, 110.0]))
    u = np.linspace(-1, 1, 9)
    for ai, wii in zip(a, wi):
        assert np.allclose(U.model_density(u, ai, wii), 0.5, rtol=1e-12)


def test_run_with_urban_scatter_closes_the_ledger():
    """A 20-step run on gold with the Urban-type model: the ledger closes,
    electrons are turned (differently from Davies, same draws), and more
    of them turn back through large angles than with Davies."""
    base = dict(nx=16, ny=12, nz=12, x_lo=2e-6, x_hi=14e-6, physics=W.PHYS_ALL & ~W.PHYS_FIELDS,
                max_particles=20000, series_len=20)
    src = W.source(n_macro=2000, y0=6e-6, z0=6e-6, r_fwhm=4e-6, T_hot=1 * MEV, t_end=0.1e-12)
    runs = {}
    for name, extra in (("davies", 0), ("urban", R.PHYS_URBAN)):
        cfg = W.base_config(**dict(base, physics=base["physics"] | extra))
        r = OracleRun(cfg)
        r.add_source(src)
        r.run(20)
        runs[name] = r
    d, u = runs["davies"], runs["urban"]
    assert u.closure() < 1e-12
    assert not np.allclose(d.state()["p"][:50], u.state()["p"][:50], rtol=1e-3, atol=0.0)
    back = {k: float(np.mean(r.p[:, 0] < 0)) for k, r in runs.items()}
    print(f"  fraction moving back: {back}")
    assert back["urban"] > back["davies"]


def test_urban_needs_the_scatter_bit():
    with pytest.raises(ValueError):
        OracleRun(W.base_config(physics=R.PHYS_ION | R.PHYS_URBAN))
