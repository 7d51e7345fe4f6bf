"""Background solid: ionisation state, Coulomb logarithm, reduced Lee-More
resistivity, heat capacity, Ohmic + ionisation heating and electron-ion
exchange (App. A of the paper).  Oracle-only implementation, FP64, SI,
temperatures in kelvin.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as K


def ion_density(rho: float, A: float) -> float:
    """n_i [m^-3] of a solid of mass density rho [kg/m^3] and molar mass A [g/mol]."""
    return rho / (A * K.AMU)


def zstar_more(Z, A, rho, Te):
    """Ionisation state Z*.  The paper cites More's Table IV algorithm without
    printing it; this is More's published Thomas-Fermi fit (temperature in
    eV, density in g/cm^3).  PARITY UNPINNED in absolute value: only its
    limits (0 < Z* <= Z, Z* -> Z when hot, monotone in T) are pinned."""
    T_ev = np.asarray(Te, dtype=np.float64) * K.KB / K.E
    alpha, beta = 14.3139, 0.6624
    a1, a2, a3, a4 = 0.003323, 0.971832, 9.26148e-5, 3.10165
    b0, b1, b2 = -1.7630, 1.43175, 0.31546
    c1, c2 = -0.366667, 0.983333
    R = (rho * 1e-3) / (A * Z)              # g/cm^3 per (A Z)
    T0 = T_ev / Z ** (4.0 / 3.0)
    Tf = T0 / (1.0 + T0)
    Acoef = a1 * T0 ** a2 + a3 * T0 ** a4
    Bcoef = -np.exp(b0 + b1 * Tf + b2 * Tf ** 7)
    Ccoef = c1 * Tf + c2
    Q1 = Acoef * R ** Bcoef
    Q = (R ** Ccoef + Q1 ** Ccoef) ** (1.0 / Ccoef)
    x = alpha * Q ** beta
    return Z * x / (1.0 + x + np.sqrt(1.0 + 2.0 * x))


def coulomb_log(Te, Ti, Zs, n_i):
    """ln Lambda.  The paper cites the Lee-More method without printing it.
    Reading: ln L = max(2, 0.5 ln(1 + (b_max/b_min)^2)) with
      b_max = max(lambda_D, R0), R0 = (3/(4 pi n_i))^(1/3),
      lambda_D^-2 = e^2 n_e/(eps0 kB T_eff) + Z*^2 e^2 n_i/(eps0 kB T_i),
      T_eff = sqrt(T_e^2 + T_F^2), kB T_F = hbar^2 (3 pi^2 n_e)^(2/3)/(2 m_e),
      b_min = max(Z* e^2/(12 pi eps0 kB T_eff), hbar/(2 sqrt(3 m_e kB T_eff))),
    with n_e = Z* n_i.  PARITY UNPINNED in absolute value."""
    Te = np.asarray(Te, dtype=np.float64)
    Ti = np.asarray(Ti, dtype=np.float64)
    ne = Zs * n_i
    TF = K.HBAR ** 2 * (3.0 * math.pi ** 2 * ne) ** (2.0 / 3.0) / (2.0 * K.ME * K.KB)
    Teff = np.sqrt(Te * Te + TF * TF)
    inv_ld2 = K.E ** 2 * ne / (K.EPS0 * K.KB * Teff) + Zs ** 2 * K.E ** 2 * n_i / (K.EPS0 * K.KB * Ti)
    lam_d = 1.0 / np.sqrt(inv_ld2)
    R0 = (3.0 / (4.0 * math.pi * n_i)) ** (1.0 / 3.0)
    bmax = np.maximum(lam_d, R0)
    bmin = np.maximum(Zs * K.E ** 2 / (12.0 * math.pi * K.EPS0 * K.KB * Teff),
                      K.HBAR / (2.0 * np.sqrt(3.0 * K.ME * K.KB * Teff)))
    return np.maximum(2.0, 0.5 * np.log(1.0 + (bmax / bmin) ** 2))


def tau_hot(Te, Zs, n_i, lnL):
    """(tau A^alpha)_hot = 128 pi eps0^2/(3 e^4) sqrt(m_e/(2 pi)) (kB Te)^(3/2)/(Z*^2 n_i lnL)."""
    kT = K.KB * np.asarray(Te, dtype=np.float64)
    return (128.0 * math.pi * K.EPS0 ** 2 / (3.0 * K.E ** 4) * math.sqrt(K.ME / (2.0 * math.pi))
            * kT ** 1.5 / (Zs ** 2 * n_i * lnL))


def tau_cold(Te, n_i, lambda1):
    """(tau A^alpha)_cold = lambda1 R0 / vbar, vbar = sqrt(3 kB Te / m_e)."""
    R0 = (3.0 / (4.0 * math.pi * n_i)) ** (1.0 / 3.0)
    vbar = np.sqrt(3.0 * K.KB * np.asarray(Te, dtype=np.float64) / K.ME)
    return lambda1 * R0 / vbar


def resistivity(Te, Ti, Z, A, rho, lambda1, lambda2):
    """Reduced Lee-More resistivity eq. (LeeMoreGeneral) times lambda2:
    eta = lambda2 m_e / (Z* n_i e^2 max(tau_hot, tau_cold)).  Returns
    (eta, Z*, lnL)."""
    n_i = ion_density(rho, A)
    Zs = zstar_more(Z, A, rho, Te)
    lnL = coulomb_log(Te, Ti, Zs, n_i)
    tau = np.maximum(tau_hot(Te, Zs, n_i, lnL), tau_cold(Te, n_i, lambda1))
    return lambda2 * K.ME / (Zs * n_i * K.E ** 2 * tau), Zs, lnL


def heat_capacity(Te, Z):
    """C = 0.3 + 1.2 T'(2.2 + T')/(1.1 + T')^2, T' = (kB Te / e) Z^-4/3 (App. A)."""
    Tp = K.KB * np.asarray(Te, dtype=np.float64) / K.E * Z ** (-4.0 / 3.0)
    return 0.3 + 1.2 * Tp * (2.2 + Tp) / (1.1 + Tp) ** 2


def exchange_rates(Te, Ti, Zs, lnL, n_i, m_i):
    """Rates (a, b) [1/s] of the electron-ion exchange of App. A:
    dTe/dt = a (Ti - Te), dTi/dt = b (Te - Ti), with a = Z*^2 e^4 n_i / t_c,
    b = Z*^3 e^4 n_i / t_c and
    1/t_c = 2/(3 (2 pi kB)^(3/2)) sqrt(m_e m_i) lnL / (eps0^2 (Te m_i + Ti m_e)^(3/2))."""
    inv_tc = (2.0 / (3.0 * (2.0 * math.pi * K.KB) ** 1.5) * math.sqrt(K.ME * m_i) * lnL
              / (K.EPS0 ** 2 * (Te * m_i + Ti * K.ME) ** 1.5))
    a = Zs ** 2 * K.E ** 4 * n_i * inv_tc
    b = Zs ** 3 * K.E ** 4 * n_i * inv_tc
    return a, b


def exchange_exact(Te, Ti, a, b, dt):
    """Exact solution of the linear exchange over dt with frozen rates:
    M = (b Te + a Ti)/(a + b) is conserved, Te - Ti decays as exp(-(a+b) dt)."""
    s = a + b
    M = (b * Te + a * Ti) / s
    D = (Te - Ti) * np.exp(-s * dt)
    return M + a / s * D, M - b / s * D


def heat_update(Te, Ti, j2, ion_heat, eta, dt, dV, Z, A, rho, lambda1, lambda2):
    """One temperature/resistivity update of solid cells (App. A):
      rho_eps = eta |j_h|^2 dt + (ionisation energy)/dV
      Te += rho_eps / (Z n_i C(Te) kB)             eq. (Te_rise)
      electron-ion exchange over dt, rates frozen at (Te, Ti, Z*(Te))
      eta, Z*, lnL from the final temperatures.
    j2 = |j_h|^2 at the cell centre [A^2/m^4], ion_heat [J] per cell.
    Returns (Te, Ti, eta)."""
    n_i = ion_density(rho, A)
    m_i = A * K.AMU
    rho_eps = eta * j2 * dt + ion_heat / dV
    C = heat_capacity(Te, Z)
    Te1 = Te + rho_eps / (Z * n_i * C * K.KB)
    Zs1 = zstar_more(Z, A, rho, Te1)
    lnL1 = coulomb_log(Te1, Ti, Zs1, n_i)
    a, b = exchange_rates(Te1, Ti, Zs1, lnL1, n_i, m_i)
    Te2, Ti2 = exchange_exact(Te1, Ti, a, b, dt)
    eta2, _, _ = resistivity(Te2, Ti2, Z, A, rho, lambda1, lambda2)
    return Te2, Ti2, eta2


def f_sigma(Te, Ti, Z, A, rho):
    """Enhancement factor of the bremsstrahlung cross-sections by the
    ionisation of the background (eq. F_sigma, Sec. II.B):
      F = 1 + ln|lambda_D / a_s| / ln|a_s m_e c / hbar| (Z*/Z)^2,
    lambda_D the Debye length of the background ions,
    lambda_D^-2 = Z*^2 e^2 n_i / (eps0 kB Ti), a_s = 1.4 a_B Z^(-1/3).
    Reading: the printed ln|a_s m_e c^2 / hbar| is not dimensionless; with
    m_e c (a_s over the reduced Compton wavelength) it is the complete-
    screening logarithm ln(192 Z^(-1/3)), so a fully ionised cell has the
    ratio of the two screening logarithms, ln(lambda_D/lbar_C)/ln(a_s/lbar_C)."""
    Te = np.asarray(Te, dtype=np.float64)
    Ti = np.asarray(Ti, dtype=np.float64)
    n_i = ion_density(rho, A)
    Zs = zstar_more(Z, A, rho, Te)
    lam = np.sqrt(K.EPS0 * K.KB * Ti / (Zs * Zs * K.E * K.E * n_i))
    a_s = 1.4 * K.A_BOHR * Z ** (-1.0 / 3.0)
    return 1.0 + np.log(np.abs(lam / a_s)) / np.log(abs(a_s * K.ME * K.C / K.HBAR)) * (Zs / Z) ** 2


def n_sub_auto(dt, dx, Z, A, rho, T0, lambda1, lambda2):
    """Field sub-cycles for the explicit resistive diffusion of
    eqs. (Ampere_Maxwell, Faraday_Lens): stable for dt_sub <= mu0 dx^2/(6 eta).
    eta_max is the largest resistivity on 400 log-spaced equal temperatures
    from T0 to 1e9 K; dt_sub = 0.9 mu0 dx^2/(6 eta_max)."""
    T = np.logspace(math.log10(T0), 9.0, 400)
    eta, _, _ = resistivity(T, T, Z, A, rho, lambda1, lambda2)
    dt_max = 0.9 * K.MU0 * dx * dx / (6.0 * float(np.max(eta)))
    return max(1, int(math.ceil(dt / dt_max)))


# ---------------------------------------------------------------------------
# compound solids (App. A: several single-element solids in one cell)
# ---------------------------------------------------------------------------
# An element of a compound is a dict with Z, A [g/mol], rho (its partial mass
# density [kg/m^3]) and n (its ion density [m^-3]).  The paper gives the rule
# for the electron heating only: n_e = Z n_i of eq. Te_rise becomes the sum of
# Z n over the solids, and 1/C is averaged with weights Z n.  Readings for
# the rest, chosen so that two overlapping halves of one material behave as
# that material (the paper's stated criterion for its heating rule):
#   * each element's Z*, Coulomb logarithm, relaxation time and resistivity are
#     evaluated as if the element filled the cell at the total ion density
#     n_t = sum n (for Z*: at the mass density n_t A amu);
#   * resistivity: the free electrons' collision rates add over the ion
#     species in proportion to their shares x = n / n_t (Matthiessen), so
#     eta = sum(x Z* eta_el) / sum(x Z*);
#   * exchange: dTe/dt = (Ti - Te) sum(x a_el), and energy conservation
#     between n_e* = n_t sum(x Z*) free electrons and n_t ions gives
#     dTi/dt = (Te - Ti) sum(x a_el) sum(x Z*).
# With one element all of these are the single-element formulas above.

def element(Z, A, rho):
    return dict(Z=float(Z), A=float(A), rho=float(rho), n=ion_density(rho, A))


def heat_capacity_mix(Te, elems):
    """<1/C> weighted by Z n (App. A compounds) and n_e = sum Z n: returns
    (n_e, <1/C>)."""
    ne = sum(e["Z"] * e["n"] for e in elems)
    inv_c = sum(e["Z"] * e["n"] / heat_capacity(Te, e["Z"]) for e in elems) / ne
    return ne, inv_c


def _as_if_filled(e, n_t):
    """The element as if it filled the cell at the total ion density."""
    return dict(e, n=n_t, rho=n_t * e["A"] * K.AMU)


def resistivity_mix(Te, Ti, elems, lambda1, lambda2):
    """Compound resistivity (reading above).  Returns (eta, [Z*_el], [lnL_el])."""
    n_t = sum(e["n"] for e in elems)
    num, den = 0.0, 0.0
    zs, lls = [], []
    for e in elems:
        f = _as_if_filled(e, n_t)
        eta_e, Zs, lnL = resistivity(Te, Ti, f["Z"], f["A"], f["rho"], lambda1, lambda2)
        x = e["n"] / n_t
        num = num + x * Zs * eta_e
        den = den + x * Zs
        zs.append(Zs)
        lls.append(lnL)
    return num / den, zs, lls


def heat_update_mix(Te, Ti, j2, ion_heat, eta, dt, dV, elems, lambda1, lambda2):
    """heat_update for a compound: the heating of eq. Te_rise with the
    paper's compound rule, exchange and resistivity by the readings above."""
    n_t = sum(e["n"] for e in elems)
    rho_eps = eta * j2 * dt + ion_heat / dV
    ne, inv_c = heat_capacity_mix(Te, elems)
    Te1 = Te + rho_eps * inv_c / (ne * K.KB)
    a = 0.0
    zbar = 0.0
    for e in elems:
        f = _as_if_filled(e, n_t)
        Zs = zstar_more(f["Z"], f["A"], f["rho"], Te1)
        lnL = coulomb_log(Te1, Ti, Zs, n_t)
        a_e, _ = exchange_rates(Te1, Ti, Zs, lnL, n_t, f["A"] * K.AMU)
        x = e["n"] / n_t
        a = a + x * a_e
        zbar = zbar + x * Zs
    Te2, Ti2 = exchange_exact(Te1, Ti, a, a * zbar, dt)
    eta2, _, _ = resistivity_mix(Te2, Ti2, elems, lambda1, lambda2)
    return Te2, Ti2, eta2


def n_sub_auto_mix(dt, dx, elems, T0, lambda1, lambda2):
    """n_sub_auto with the compound resistivity."""
    T = np.logspace(math.log10(T0), 9.0, 400)
    eta, _, _ = resistivity_mix(T, T, elems, lambda1, lambda2)
    dt_max = 0.9 * K.MU0 * dx * dx / (6.0 * float(np.max(eta)))
    return max(1, int(math.ceil(dt / dt_max)))
