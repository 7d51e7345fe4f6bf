"""Urban-type elastic scatter (App. B): model functions for the polar angle
after one step whose first two angular moments are those of Lewis theory.
Oracle-only implementation, FP64, SI; test infrastructure, never called by
the product path.

The paper adopts, as its alternative to the Davies model, Urban's approach:
the deflection of a step is drawn from model functions whose moments match
Lewis theory, with no spatial displacement inside the step (steps stay
within one cell).  It prints neither the model functions nor the transport
cross-sections, so everything below is a reading (each also listed with the
design notes):

  * Lewis theory: for a path s, <P_l(cos theta)> = exp(-s / lambda_l), with
    1 / lambda_l = sum over elements of n sigma_l, sigma_l the transport
    cross-section with weight 1 - P_l(cos chi).  s = v dt.
  * Single scattering: the screened Rutherford (Wentzel) cross-section
    d sigma / d Omega = k / (mu + A)^2, mu = (1 - cos chi) / 2,
    k = Z (Z + 1) r_e^2 (m c^2)^2 / (4 (p v)^2) (nucleus and atomic
    electrons), Moliere's screening parameter
    A = (hbar / (2 p a_TF))^2 (1.13 + 3.76 (alpha Z / beta)^2),
    a_TF = 0.88534 a_0 Z^(-1/3).  Integrated over d Omega = 4 pi d mu:
      sigma_1 = 8 pi k (ln(1 + 1/A) - 1 / (1 + A))
      sigma_2 = 24 pi k ((1 + 2 A) ln(1 + 1/A) - 2)
  * Model function of u = cos theta on [-1, 1]: a core
    f1(u) = a exp(-a (1 - u)) / (1 - exp(-2 a)) with weight 1 - w_i and an
    isotropic part 1/2 with weight w_i.  The core's Legendre moments are
    L(a) = coth a - 1/a and 1 - 3 L(a) / a, the isotropic part's are zero,
    so matching both Lewis moments q_1 = exp(-x_1), q_2 = exp(-x_2)
    (x_l = s / lambda_l) gives one equation for a,
      1 / L(a) - 3 / a = q_2 / q_1,
    whose left side rises from 0 (a -> 0) to 1 (a -> infinity), and then
    w_i = 1 - q_1 / L(a).  Where that w_i would be negative (a few long
    steps of slow electrons), w_i = 0 and a matches the first moment alone,
    L(a) = q_1.  Urban's fitted corrections to the central width (his
    empirical fit to scattering data) are not in the paper and not used.
  * Draws: the slot of the Davies model; the first uniform picks the part
    (isotropic when it is below w_i), the second gives 1 - u by the inverse
    CDF of the part, the third the azimuth.

Parity pinned by: the transport cross-sections against quadrature of the
single-scattering law; the mixture's moments, by quadrature of its density,
against the Lewis values; the sampler's moments and its CDF; the small-step
limit against the Davies variance; large steps tend to isotropy.
"""
from __future__ import annotations

import math

from fractions import Fraction

import numpy as np
from mpmath import bernfrac

from . import constants as K
from . import particles as PT

TF = 0.88534              # Thomas-Fermi radius in units of a_0 Z^(-1/3)
M_C1, M_C2 = 1.13, 3.76   # Moliere's screening constants

# coth a - 1/a = sum_{n >= 1} 2^(2n) B_2n a^(2n-1) / (2n)!  (|a| < pi), with
# the Bernoulli numbers as exact fractions
_NSER = 20
_LCOEF = np.array([float(Fraction(2 ** (2 * n)) * Fraction(*bernfrac(2 * n)) / math.factorial(2 * n))
                   for n in range(1, _NSER + 1)])
_SMALL = 1.0              # below: the series, above: the closed form


def screening(um, beta, Z):
    """Moliere's screening parameter A of momentum u = p/(m c) (the
    reduced Compton wavelength hbar/(m c) is alpha a_0)."""
    return (K.ALPHA * Z ** (1.0 / 3.0) / (2.0 * TF * um)) ** 2 * (M_C1 + M_C2 * (K.ALPHA * Z / beta) ** 2)


def transport_xs(eps, Z):
    """(sigma_1, sigma_2) per atom [m^2] of an electron of kinetic energy
    eps [J] in element Z, from the screened Rutherford law."""
    eps = np.asarray(eps, dtype=np.float64)
    g = 1.0 + eps / K.MEC2
    um = np.sqrt(g * g - 1.0)
    beta = um / g
    A = screening(um, beta, Z)
    k = Z * (Z + 1.0) * K.R_E ** 2 / (4.0 * (um * beta) ** 2)
    lg = np.log1p(1.0 / A)
    return (8.0 * math.pi * k * (lg - 1.0 / (1.0 + A)),
            24.0 * math.pi * k * ((1.0 + 2.0 * A) * lg - 2.0))


def lewis_x(eps, elems, dt):
    """x_1 = s / lambda_1 and x_2 = s / lambda_2 of one step, s = v dt,
    summed over the elements (each a dict with Z and n)."""
    eps = np.asarray(eps, dtype=np.float64)
    g = 1.0 + eps / K.MEC2
    s = np.sqrt(1.0 - 1.0 / (g * g)) * K.C * dt
    x1 = np.zeros_like(eps)
    x2 = np.zeros_like(eps)
    for e in elems:
        s1, s2 = transport_xs(eps, e["Z"])
        x1 = x1 + e["n"] * s1 * s
        x2 = x2 + e["n"] * s2 * s
    return x1, x2


def langevin(a):
    """L(a) = coth a - 1/a: the series below 1, the closed form above."""
    a = np.asarray(a, dtype=np.float64)
    small = a < _SMALL
    out = np.empty_like(a)
    aa = a[small]
    out[small] = sum(c * aa ** (2 * n + 1) for n, c in enumerate(_LCOEF))
    ab = a[~small]
    with np.errstate(over="ignore"):
        out[~small] = 1.0 - (1.0 / ab - 2.0 / np.expm1(2.0 * ab))
    return out


def _one_minus_langevin(a):
    """1 - L(a), accurate for large a: 1/a - 2/(e^(2a) - 1)."""
    a = np.asarray(a, dtype=np.float64)
    with np.errstate(over="ignore"):
        big = 1.0 / a - 2.0 / np.expm1(2.0 * a)
    return np.where(a < _SMALL, 1.0 - langevin(np.minimum(a, _SMALL)), big)


def _phi_small(a):
    """1/L(a) - 3/a for a < 1, as (a - 3 L(a)) / (a L(a)) with the series'
    first term (a/3) cancelled exactly."""
    rest = sum(c * a ** (2 * n + 1) for n, c in enumerate(_LCOEF) if n > 0)
    return -3.0 * rest / (a * langevin(a))


def _bisect(F, n, lo=-40.0, hi=40.0, iters=70):
    """Root in ln a of a decreasing residual F(a) (vectorised bisection)."""
    lo = np.full(n, lo)
    hi = np.full(n, hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pos = F(np.exp(mid)) > 0.0
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
    return np.exp(0.5 * (lo + hi))


def model_params(x1, x2):
    """Core parameter a and isotropic weight w_i matching the Lewis moments
    exp(-x_1), exp(-x_2) (w_i = 0 and the first moment alone where the
    match needs w_i < 0)."""
    x1 = np.atleast_1d(np.asarray(x1, dtype=np.float64))
    x2 = np.atleast_1d(np.asarray(x2, dtype=np.float64))
    n = len(x1)
    d = x2 - x1
    r = np.exp(-d)              # q_2 / q_1
    rho = -np.expm1(-d)         # 1 - q_2 / q_1

    def F(a):                   # 1 - (1/L - 3/a) - rho, decreasing in a
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            c1 = _one_minus_langevin(a)
            big = 3.0 / a - c1 / (1.0 - c1) - rho
            small = r - _phi_small(np.minimum(a, _SMALL))
        return np.where(a < _SMALL, small, big)

    a = _bisect(F, n)
    om = -np.expm1(-x1)         # 1 - q_1
    c1 = _one_minus_langevin(a)
    wi = (om - c1) / langevin(a)   # 1 - q_1 / L(a), as differences from 1
    bad = wi < 0.0
    if np.any(bad):
        omb = om[bad]

        def F1(aa):              # (1 - L(a)) - (1 - q_1), decreasing in a
            return _one_minus_langevin(aa) - omb

        a[bad] = _bisect(F1, int(np.sum(bad)))
        wi[bad] = 0.0
    return a, wi


def one_minus_cos(a, wi, ua, ub):
    """1 - cos theta drawn from the model function: isotropic (2 (1 - ub))
    when ua < w_i, else the core's inverse CDF
    -ln(1 - (1 - ub)(1 - exp(-2a))) / a."""
    iso = 2.0 * (1.0 - ub)
    core = -np.log1p(-(1.0 - ub) * -np.expm1(-2.0 * a)) / a
    return np.where(ua < wi, iso, core)


def model_density(u, a, wi):
    """Density of u = cos theta on [-1, 1] (for the quadrature pins)."""
    core = a * np.exp(-a * (1.0 - u)) / -np.expm1(-2.0 * a)
    return (1.0 - wi) * core + 0.5 * wi


def scatter(p, elems, dt, ua, ub, uc):
    """Momenta after one step of Urban-type elastic scatter: the polar
    angle from the model function of the step, a uniform azimuth 2 pi uc."""
    eps = PT.kinetic(p)
    x1, x2 = lewis_x(eps, elems, dt)
    a, wi = model_params(x1, x2)
    w = one_minus_cos(a, wi, ua, ub)
    th = 2.0 * np.arcsin(np.sqrt(0.5 * w))
    return PT.rotate(p, th, 2.0 * math.pi * uc)
