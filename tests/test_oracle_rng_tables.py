"""Oracle pins: the counter-based generator and the bremsstrahlung tables.

Each test fixes a part of the oracle against something other than the oracle
itself: published known-answer vectors, numerical quadrature of the spectral
shape, or the paper's printed stopping-power formula.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import constants as K
from oracle import philox as P
from oracle import tables as T


def test_philox_known_answers(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append(v)
    assert len(rows) == 3
    for v in rows:
        out = P.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_uniform_mapping_exact_and_open():
    # extremes of the 32-bit range map strictly inside (0, 1), exactly in FP32
    u = P.to_uniform(np.array([0, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] > 0.0 and u[1] < 1.0
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert u[0] == 0.5 * 2.0 ** -23 and u[1] == 1.0 - 0.5 * 2.0 ** -23


def test_uniforms_distribution_and_independence():
    ids = np.arange(200000)
    u = P.uniforms(ids, 7, 3, 0)
    for c in u:
        assert stats.kstest(c, "uniform").pvalue > 1e-3
    # different slots, steps and seeds give unrelated streams
    v = P.uniforms(ids, 7, 3, 1)[0]
    w = P.uniforms(ids, 8, 3, 0)[0]
    assert abs(np.corrcoef(u[0], v)[0, 1]) < 0.01
    assert abs(np.corrcoef(u[0], w)[0, 1]) < 0.01


# --------------------------------------------------------------------------
# tables
# --------------------------------------------------------------------------
def test_cz_equals_printed_stop_brem_prefactor(golden_dir):
    """eq. (stop_brem): gamma e^6/(12 pi^3 eps0^3 m c^3 hbar) n_i Z^2 ln(5.6 pi eps0 hbar c/(Z^1/3 e^2)).
    The oracle's C_Z per unit energy must equal that expression divided by gamma m c^2 n_i."""
    for Z in (13.0, 29.0, 79.0):
        printed = (K.E ** 6 / (12 * math.pi ** 3 * K.EPS0 ** 3 * K.ME * K.C ** 3 * K.HBAR) * Z * Z
                   * math.log(5.6 * math.pi * K.EPS0 * K.HBAR * K.C / (Z ** (1 / 3) * K.E ** 2)))
        assert T.c_z(Z) * K.MEC2 == pytest.approx(printed, rel=1e-12)


@pytest.mark.parametrize("shape", [T.CSBH, T.FLAT])
@pytest.mark.parametrize("eps_mev", [0.003, 0.1, 1.0, 30.0, 800.0])
def test_sigma_and_subcut_by_quadrature(shape, eps_mev):
    k_cut = 1e3 * K.E
    eps = eps_mev * 1e6 * K.E
    # spectral shape written out independently: k dsigma/dk / C_Z
    if shape == T.CSBH:
        kds = lambda k: 4.0 / 3.0 * (1 - k / eps) + (k / eps) ** 2
    else:
        kds = lambda k: 1.0
    sig_q = integrate.quad(lambda lk: kds(math.exp(lk)), math.log(k_cut), math.log(eps),
                           epsabs=0, epsrel=1e-12)[0]
    sub_q = integrate.quad(lambda k: kds(k), 0.0, min(k_cut, eps), epsabs=0, epsrel=1e-12)[0]
    assert float(T.sigma_norm(eps, k_cut, shape)) == pytest.approx(sig_q, rel=1e-9)
    assert float(T.sub_norm(eps, k_cut, shape)) == pytest.approx(sub_q, rel=1e-9)
    # the full spectrum integrates to eps: the radiative stopping of eq. (stop_brem)
    tot = integrate.quad(lambda k: kds(k), 0.0, eps, epsabs=0, epsrel=1e-12, limit=200)[0]
    assert tot == pytest.approx(eps, rel=1e-9)


@pytest.fixture(scope="module")
def tab():
    return T.BremTable(1e3 * K.E, 10e9 * K.E, 128, 256, T.CSBH)


def test_inverse_cdf_nodes_by_quadrature(tab):
    """At table nodes, x(r) must satisfy F(x) = r where F is the quadrature of the
    shape between k_cut and k(x)."""
    k_cut = tab.k_cut
    for j in (1, 17, 64, 127):
        eps = tab.eps[j]
        tot = integrate.quad(lambda lk: 4 / 3 * (1 - math.exp(lk) / eps) + (math.exp(lk) / eps) ** 2,
                             math.log(k_cut), math.log(eps), epsrel=1e-12)[0]
        for i in (13, 128, 250):
            x = tab.X[j, i]
            k = k_cut * (eps / k_cut) ** x
            part = integrate.quad(lambda lk: 4 / 3 * (1 - math.exp(lk) / eps) + (math.exp(lk) / eps) ** 2,
                                  math.log(k_cut), math.log(k), epsrel=1e-12)[0]
            assert part / tot == pytest.approx(tab.r[i], abs=1e-10)


def test_table_radiative_stopping_matches_stop_brem(tab):
    """Integrating the tabulated cross-section: sigma(eps) <k> + S_sub(eps) = eps,
    i.e. n_i C_Z eps -- eq. (stop_brem) with gamma m c^2 -> eps -- within the
    table's interpolation error."""
    r = (np.arange(20000) + 0.5) / 20000
    for eps_mev in (0.05, 0.5, 3.0, 40.0, 500.0):
        eps = eps_mev * 1e6 * K.E
        kmean = np.mean(tab.sample_k(np.full_like(r, eps), r))
        total = tab.sigma(eps) * kmean + tab.sub(eps)
        assert float(total) == pytest.approx(eps, rel=2e-3)


def test_table_sampling_matches_exact_cdf(tab):
    """Between rows, the sampled x follows the exact CDF to the interpolation error."""
    eps = 7.3e6 * K.E              # not a table node
    r = (np.arange(4000) + 0.5) / 4000
    x = tab.sample_x(np.full_like(r, eps), r)
    F = T.cdf_x(x, eps, tab.k_cut, T.CSBH)
    assert np.max(np.abs(F - r)) < 2e-3


def test_flat_table_gives_uniform_log_energy():
    tab = T.BremTable(1e3 * K.E, 10e9 * K.E, 64, 128, T.FLAT)
    rng = np.random.default_rng(1)
    r = rng.random(50000)
    eps = 2.0e6 * K.E
    k = tab.sample_k(np.full_like(r, eps), r)
    x = np.log(k / tab.k_cut) / math.log(eps / tab.k_cut)
    assert stats.kstest(x, "uniform").pvalue > 1e-3
    assert np.all((k >= tab.k_cut * (1 - 1e-12)) & (k <= eps * (1 + 1e-12)))
