"""The paper's simple energy-partition model (Sec. III.B): the exponential
injection condensed into three macro-electrons ("warm" below the X-ray
threshold, "emitting" up to the escape energy, "escaping" above it), each
integrated through four continuous stopping powers -- bremsstrahlung eq.
(stop_brem), ionisation eq. (stop_ion), reflux eq. (stop_tnsa) and the
resistive field eq. (stop_field).  Oracle-only implementation, FP64, SI;
test infrastructure, never called by the product path.

Readings where the paper is silent (also listed with the design notes):
  * bins: warm [0, e1), emitting [e1, e_esc), escaping [e_esc, inf) with
    e1 = min(e_th, e_esc) (the emitting bin is empty when e_esc <= e_th);
  * the photon stopping above the threshold is eq. stop_brem evaluated at
    the kinetic energy eps - e_th (zero below the threshold); it is part of
    the bremsstrahlung loss, not a fifth mechanism;
  * x in eq. stop_field is the path length travelled;
  * the warm and emitting macro-electrons run until their energy is spent;
    the escaping one until its path reaches L_x, where what it has not lost
    escapes (all of it is absorbed if it is spent first);
  * the integration: classical fourth-order Runge-Kutta with the energy as
    the independent variable, n uniform steps of u = ln(1 + eps / eps_s),
    eps_s = 1 keV, from the macro-electron's energy down to zero; the state
    is the path x and the energy given to each mechanism.  The escaping
    electron's state at L_x is the linear interpolation in x between the two
    steps around the crossing.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as K
from . import particles as PT

EPS_S = 1e3 * K.E      # energy scale of the integration variable [J]
OUT_KEYS = ("brem", "photon_thr", "ionisation", "reflux", "field", "escaped")


def a0_of(I0, wavelength):
    """eq. a0."""
    return 8.5e-6 * np.sqrt(I0 * wavelength ** 2)


def macro_electrons(T, e_th, e_esc, N):
    """Electron counts W and total kinetic energies E of the three
    macro-electrons: integrals of dN/de = N/T exp(-e/T) and of e dN/de over
    the three bins.  T, e_th, e_esc, N broadcast; returns arrays [3, ...]."""
    T, e_th, e_esc, N = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (T, e_th, e_esc, N)))
    e1 = np.minimum(e_th, e_esc)
    edges = [np.zeros_like(T), e1, e_esc, np.full_like(T, np.inf)]
    cn = [1.0 - np.exp(-e / T) for e in edges]                    # N fraction below e
    ce = [T - (e + T) * np.exp(-e / T) for e in edges[:3]] + [T]  # energy / N below e
    W = np.array([N * (cn[k + 1] - cn[k]) for k in range(3)])
    E = np.array([N * (ce[k + 1] - ce[k]) for k in range(3)])
    return W, E


def params(m, I0, Z):
    """Constants of scan points (arrays I0 [W/m^2], Z) for the model inputs m."""
    I0 = np.asarray(I0, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    a0 = a0_of(I0, m["wavelength"])
    T = a0 * K.MEC2 * m["sqrt_fg_mean"]
    n_i = np.full_like(I0, m["n_i"])
    N = (I0 * m["fg_mean"] * (math.pi * m["r_fwhm"] ** 2 / 4.0)
         * (m["t_fwhm"] * math.sqrt(math.log(10.0) / math.log(2.0))) * m["eta_l2e"] / T)
    k_brem = (K.E ** 6 / (12.0 * math.pi ** 3 * K.EPS0 ** 3 * K.ME * K.C ** 3 * K.HBAR) * n_i * Z * Z
              * np.log(5.6 * math.pi * K.EPS0 * K.HBAR * K.C / (Z ** (1.0 / 3.0) * K.E ** 2)))
    L = m["Lx"] + m["Ly"] + m["Lz"]
    return dict(a0=a0, T=T, N=N, Z=Z, n_i=n_i, I_ex=11.0 * K.E * Z, e_th=np.full_like(I0, m["e_th"]),
                e_esc=m["kappa_esc"] * a0 * K.MEC2, k_brem=k_brem,
                s_tnsa=3.0 * m["kappa_tnsa"] * a0 * K.MEC2 / L,
                k_field=(K.E ** 2 * m["eta_mean"] * I0 * m["fg_mean"] * (0.5 * m["r_fwhm"]) ** 2
                         * m["eta_l2e"] / T),
                tan_c=math.tan(m["theta_c"]), r_half=0.5 * m["r_fwhm"], Lx=m["Lx"])


def stopping(eps, x, p):
    """Stopping powers [J/m] at kinetic energies eps and paths x (arrays):
    bremsstrahlung eq. stop_brem, its part from photons above e_th,
    ionisation eq. stop_ion (zero at eps = 0), reflux eq. stop_tnsa and the
    field eq. stop_field."""
    g = 1.0 + eps / K.MEC2
    brem = p["k_brem"] * g
    thr = np.where(eps > p["e_th"], p["k_brem"] * (1.0 + (eps - p["e_th"]) / K.MEC2), 0.0)
    mom = np.zeros(np.shape(eps) + (3,))
    mom[..., 0] = PT.momentum_of_energy(eps)
    with np.errstate(divide="ignore", invalid="ignore"):
        ion = PT.stopping_ion(eps, mom, p["Z"], p["n_i"], p["I_ex"])
    ion = np.where(eps > 0.0, ion, 0.0)
    tnsa = p["s_tnsa"]
    field = p["k_field"] / (x * p["tan_c"] + p["r_half"]) ** 2
    return brem, thr, ion, tnsa, field


def _rhs(u, y, p):
    """d(x, E_brem, E_thr, E_ion, E_tnsa, E_field)/d(-u) per electron."""
    eps = EPS_S * np.expm1(u)
    b, t, i, r, f = stopping(eps, y[0], p)
    tot = b + i + r + f
    de = EPS_S * np.exp(u)          # d eps / d u
    return np.array([de / tot, de * b / tot, de * t / tot, de * i / tot, de * r / tot, de * f / tot])


def integrate(eps0, p, nsteps, x_stop):
    """Macro-electrons of energies eps0 (array) from x = 0 down to zero
    energy, or until the path reaches x_stop (array; inf: never).  Returns
    (losses [5, n] per electron: brem, photon_thr, ionisation, reflux, field;
    energy left where the path reached x_stop)."""
    eps0 = np.asarray(eps0, dtype=np.float64)
    u0 = np.log1p(eps0 / EPS_S)
    h = u0 / nsteps
    y = np.zeros((6,) + eps0.shape)
    u = u0.copy()
    done = np.zeros(eps0.shape, dtype=bool)
    res = np.zeros_like(y)
    left = np.zeros_like(eps0)
    for k in range(nsteps):
        # u runs from u0 down to exactly 0; the right-hand side is the rate
        # per unit of -u
        um = u0 * ((nsteps - k - 0.5) / nsteps)
        u1 = u0 * ((nsteps - k - 1.0) / nsteps)
        k1 = _rhs(u, y, p)
        k2 = _rhs(um, y + 0.5 * h * k1, p)
        k3 = _rhs(um, y + 0.5 * h * k2, p)
        k4 = _rhs(u1, y + h * k3, p)
        y1 = y + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        cross = ~done & (y1[0] >= x_stop)
        if np.any(cross):
            with np.errstate(divide="ignore", invalid="ignore"):
                s = (x_stop - y[0]) / (y1[0] - y[0])
                ys = y + s * (y1 - y)
            res[:, cross] = ys[:, cross]
            # what has not been lost escapes (photon_thr is part of brem)
            left[cross] = (eps0 - (ys[1] + ys[3] + ys[4] + ys[5]))[cross]
            done |= cross
        y, u = y1, u1
    res[:, ~done] = y[:, ~done]
    return res[1:], left


def partition(m, I0, Z, nsteps):
    """Fractions of the injected hot-electron energy at each scan point
    (arrays I0, Z): rows brem, photon_thr (eta_e->gamma), ionisation,
    reflux, field, escaped; shape [6, n]."""
    p = params(m, np.atleast_1d(I0), np.atleast_1d(Z))
    W, E = macro_electrons(p["T"], p["e_th"], p["e_esc"], p["N"])
    n = len(p["T"])
    with np.errstate(divide="ignore", invalid="ignore"):
        eps0 = np.where(W > 0.0, E / W, 0.0)                    # [3, n]
    p3 = {k: (np.broadcast_to(v, (3, n)) if np.ndim(v) else v) for k, v in p.items()}
    x_stop = np.array([np.full(n, np.inf), np.full(n, np.inf), np.full(n, m["Lx"])])
    loss, left = integrate(np.maximum(eps0, 1e-300), p3, nsteps, x_stop)
    loss = np.where(W > 0.0, loss, 0.0)
    left = np.where(W > 0.0, left, 0.0)
    out = np.concatenate([np.sum(W * loss, axis=1), [np.sum(W * left, axis=0)]])
    return out / np.sum(E, axis=0)
