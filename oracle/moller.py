"""Delta rays: discrete Moller scatter above a kinetic-energy cut and the
restricted continuous ionisation loss below it (App. B).  Oracle-only
implementation, FP64, SI; test infrastructure, never called by the product
path.

The paper splits the ionisation loss of a hot electron at the energy
eps_cut given to a background electron (1 keV in the paper):
  * below the cut, a continuous stopping power (the restricted form of App.
    B: prefactor Z n_i e^4 / (8 pi eps0^2 m v^2), logarithm
    ln(2 (gamma + 1) m^2 c^4 / I^2), plus F^- of gamma and the cut, minus the
    density effect delta);
  * above it, discrete delta rays drawn by the optical-depth method from the
    Moller cross-section, each added to the run as a new macro-electron.

F^- and the Moller cross-section come from the Moller-scatter publication
the paper cites; they are written here from their published closed forms:
  t = eps / (m c^2), D = min(eps_cut, eps / 2) / (m c^2)
  F^-(t, D) = -1 - beta^2 + ln((t - D) D) + t / (t - D)
              + (D^2 / 2 + (2 t + 1) ln(1 - D / t)) / gamma^2
  d sigma / dx = 2 pi r_e^2 Z / (beta^2 (gamma - 1))
                 [ (gamma - 1)^2 / gamma^2 + (1/x) (1/x - (2 gamma - 1)/gamma^2)
                   + (1/(1-x)) (1/(1-x) - (2 gamma - 1)/gamma^2) ]
per atom, x = energy given to the delta ray / eps, eps_cut / eps <= x <= 1/2
(the faster of the two outgoing electrons is called the primary).

Readings where the paper is silent (each also listed with the design notes):
  * delta: the paper names the density effect without a form.  Its
    high-energy limit, 2 ln(hbar omega_p / I) + 2 ln(beta gamma) - 1 with
    omega_p the plasma frequency of all Z n_i electrons, is used, clamped at
    zero (the low-energy branches of the usual parameterisation need fitted
    constants per material).
  * the energy sampler: the paper uses an unnamed published algorithm; here
    x is drawn from 1/x^2 on [x_c, 1/2] by its inverse CDF and accepted with
    probability g(x) / g_max, g = x^2 (d sigma / dx) / prefactor, which is
    convex on (0, 1/2] so g_max = max(g(x_c), g(1/2)).  At most
    N_TRIES candidates; if none is accepted the last one is taken.
  * kinematics: a free background electron at rest; energy and momentum
    conserved, the delta ray at polar angle
    cos theta = sqrt(eps_d (eps + 2 m c^2) / (eps (eps_d + 2 m c^2)))
    about the primary's direction at a uniform azimuth.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as K
from . import particles as PT
from . import philox as P

N_TRIES = 32          # rejection candidates per delta ray (16 four-draw slots)


def hbar_omega_p(Z, n_i):
    """Plasma energy of the solid's Z n_i electrons [J]."""
    return K.HBAR * math.sqrt(Z * n_i * K.E ** 2 / (K.EPS0 * K.ME))


def density_effect(bg, Z, n_i, I_ex):
    """delta(beta gamma): 2 ln(hbar omega_p / I) + 2 ln(beta gamma) - 1, >= 0."""
    bg = np.asarray(bg, dtype=np.float64)
    d = (2.0 * math.log(hbar_omega_p(Z, n_i) / I_ex)
         + 2.0 * np.log(np.maximum(bg, 1e-300)) - 1.0)
    return np.maximum(d, 0.0)


def f_minus(t, D):
    """F^-(t, D) for kinetic energy t and cut D, both in m c^2, D <= t / 2."""
    t = np.asarray(t, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    g = t + 1.0
    b2 = 1.0 - 1.0 / (g * g)
    return (-1.0 - b2 + np.log((t - D) * D) + t / (t - D)
            + (0.5 * D * D + (2.0 * t + 1.0) * np.log1p(-D / t)) / (g * g))


def restricted_stopping(eps, Z, n_i, I_ex, e_cut):
    """Restricted continuous ionisation stopping power of App. B [J/m],
    clamped >= 0; eps the kinetic energy [J], e_cut the delta-ray cut [J]."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(eps)
    ok = eps > 0.0
    t = eps[ok] / K.MEC2
    g = t + 1.0
    b2 = 1.0 - 1.0 / (g * g)
    D = np.minimum(e_cut / K.MEC2, 0.5 * t)
    lnI = math.log(I_ex / K.MEC2)
    L = (np.log(2.0 * (g + 1.0)) - 2.0 * lnI + f_minus(t, D)
         - density_effect(np.sqrt(b2) * g, Z, n_i, I_ex))
    pref = Z * n_i * K.E ** 4 / (8.0 * math.pi * K.EPS0 ** 2 * K.ME * b2 * K.C ** 2)
    out[ok] = np.maximum(pref * L, 0.0)
    return out


def restricted_stopping_mix(eps, elems, e_cut):
    """The restricted stopping power of App. B summed over the elements of a
    compound, each with its own Z n and I; the density effect is the
    compound's: omega_p of all the electrons and ln I = sum(Z n ln I)/sum(Z n).
    The total is clamped >= 0."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(eps)
    ok = eps > 0.0
    t = eps[ok] / K.MEC2
    g = t + 1.0
    b2 = 1.0 - 1.0 / (g * g)
    D = np.minimum(e_cut / K.MEC2, 0.5 * t)
    zn = sum(e["Z"] * e["n"] for e in elems)
    lnI = sum(e["Z"] * e["n"] * math.log(e["I_ex"]) for e in elems) / zn
    dens = density_effect(np.sqrt(b2) * g, zn, 1.0, math.exp(lnI))
    base = np.log(2.0 * (g + 1.0)) + f_minus(t, D) - dens
    S = 0.0
    for e in elems:
        pref = e["Z"] * e["n"] * K.E ** 4 / (8.0 * math.pi * K.EPS0 ** 2 * K.ME * b2 * K.C ** 2)
        S = S + pref * (base - 2.0 * math.log(e["I_ex"] / K.MEC2))
    out[ok] = np.maximum(S, 0.0)
    return out


def _bracket(x, g):
    a = (2.0 * g - 1.0) / (g * g)
    b = (g - 1.0) ** 2 / (g * g)
    return b + (1.0 / x) * (1.0 / x - a) + (1.0 / (1.0 - x)) * (1.0 / (1.0 - x) - a)


def moller_dxs(x, eps, Z):
    """d sigma / dx per atom [m^2] at fraction x of the kinetic energy eps [J]."""
    g = 1.0 + np.asarray(eps, dtype=np.float64) / K.MEC2
    b2 = 1.0 - 1.0 / (g * g)
    return 2.0 * math.pi * K.R_E ** 2 * Z / (b2 * (g - 1.0)) * _bracket(x, g)


def moller_sigma(eps, Z, e_cut):
    """Moller cross-section per atom for energy transfers above e_cut [m^2]:
    the integral of d sigma / dx over [x_c, 1/2], x_c = e_cut / eps; zero
    when eps <= 2 e_cut."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(eps)
    ok = eps > 2.0 * e_cut
    e = eps[ok]
    g = 1.0 + e / K.MEC2
    b2 = 1.0 - 1.0 / (g * g)
    xc = e_cut / e
    a = (2.0 * g - 1.0) / (g * g)
    b = (g - 1.0) ** 2 / (g * g)
    integral = b * (0.5 - xc) + 1.0 / xc - 1.0 / (1.0 - xc) - a * np.log((1.0 - xc) / xc)
    out[ok] = 2.0 * math.pi * K.R_E ** 2 * Z / (b2 * (g - 1.0)) * integral
    return out


def _g(x, g):
    """x^2 times the bracket of d sigma / dx."""
    return x * x * _bracket(x, g)


def sample_fraction(eps, e_cut, u):
    """Fraction x of eps given to the delta ray.  u: array [N_TRIES, 2, n] of
    uniforms, candidate k using u[k, 0] for the position and u[k, 1] for the
    acceptance."""
    eps = np.asarray(eps, dtype=np.float64)
    g = 1.0 + eps / K.MEC2
    xc = e_cut / eps
    gmax = np.maximum(_g(xc, g), _g(0.5, g))
    x = np.zeros_like(eps)
    done = np.zeros(eps.shape, dtype=bool)
    for k in range(N_TRIES):
        cand = xc / (1.0 - u[k, 0] * (1.0 - 2.0 * xc))
        acc = ~done & (u[k, 1] * gmax <= _g(cand, g))
        x = np.where(acc | (~done & (k == N_TRIES - 1)), cand, x)
        done |= acc
    return x


def sampler_uniforms(ids, seed, step):
    """The N_TRIES uniform pairs of each electron's delta ray this step: slot
    SLOT_DELTA_TRY + k // 2 holds candidates k (draws 0, 1) and k + 1 (draws
    2, 3)."""
    n = len(ids)
    u = np.empty((N_TRIES, 2, n))
    for s in range(N_TRIES // 2):
        a, b, c, d = P.uniforms(ids, seed, step, P.SLOT_DELTA_TRY + s)
        u[2 * s, 0], u[2 * s, 1], u[2 * s + 1, 0], u[2 * s + 1, 1] = a, b, c, d
    return u


def delta_kinematics(p, eps, eps_d, phi):
    """Momenta after a Moller scatter of an electron of momentum p [kg m/s]
    and kinetic energy eps on a free electron at rest, giving it eps_d:
    (primary, delta ray).  The delta ray leaves at the two-body polar angle
    at azimuth phi; the primary keeps the rest of the momentum, its length
    set from eps - eps_d."""
    cos_t = np.sqrt(eps_d * (eps + 2.0 * K.MEC2) / (eps * (eps_d + 2.0 * K.MEC2)))
    th = np.arccos(np.clip(cos_t, -1.0, 1.0))
    d = PT.rotate(p, th, phi)
    d = d * (PT.momentum_of_energy(eps_d) / np.sqrt(np.sum(d * d, axis=-1)))[:, None]
    q = p - d
    q = q * (PT.momentum_of_energy(eps - eps_d) / np.sqrt(np.sum(q * q, axis=-1)))[:, None]
    return q, d
