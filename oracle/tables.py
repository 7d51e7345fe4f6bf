"""Bremsstrahlung cross-section tables for the optical-depth emission method
(App. B of the paper).  Oracle-only implementation.

The paper samples photon energies from the Seltzer-Berger differential
cross-sections, which are data the paper does not print.  The method keeps
its mechanism here -- a tabulated total cross-section for the optical depth
and a tabulated inverse CDF for the photon energy -- filled from a closed-
form spectral shape:

  k dsigma/dk = C_Z * phi(k / eps),   0 < k <= eps  (eps = electron kinetic energy)

with C_Z = (16/3) alpha r_e^2 Z^2 ln(1.4 alpha^-1 Z^-1/3), the prefactor of
the continuous stopping power eq. (stop_brem), and one of two shapes:
  CSBH: phi(y) = 4/3 (1 - y) + y^2   (complete-screening Bethe-Heitler shape)
  FLAT: phi(y) = 1
Both integrate to 1 over y in [0, 1], so the radiative stopping power
n_i * int_0^eps k dsigma/dk dk = n_i C_Z eps reproduces eq. (stop_brem) with
the total energy gamma m c^2 replaced by the kinetic energy.

Photons below k_cut are not emitted; their energy is lost continuously at the
rate n_i S_sub(eps) v with S_sub = int_0^min(k_cut,eps) k dsigma/dk dk.

Table layout (rows in electron energy, columns in the uniform variate r):
  eps_j = k_cut (emax/k_cut)^(j/(nT-1)),  j = 0..nT-1
  r_i   = i/(nr-1),                      i = 0..nr-1
  X[j,i] = x such that F(x; eps_j) = r_i, x = ln(k/k_cut) / ln(eps/k_cut)
  SIG[j] = sigma(eps_j)/C_Z,   SUB[j] = S_sub(eps_j)/C_Z  [J]
Lookups are linear in r within a row and linear in ln(eps) between rows.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as K

CSBH = 0
FLAT = 1


def c_z(Z: float) -> float:
    """C_Z [m^2]: prefactor of eq. (stop_brem) per unit energy,
    (16/3) alpha r_e^2 Z^2 ln(1.4 alpha^-1 Z^-1/3)."""
    return (16.0 / 3.0) * K.ALPHA * K.R_E ** 2 * Z * Z * math.log(
        1.4 / K.ALPHA * Z ** (-1.0 / 3.0))


def phi(y, shape):
    y = np.asarray(y, dtype=np.float64)
    if shape == CSBH:
        return 4.0 / 3.0 * (1.0 - y) + y * y
    return np.ones_like(y)


def sigma_norm(eps, k_cut, shape):
    """sigma(eps)/C_Z = int_{k_cut}^{eps} phi(k/eps)/k dk  (0 for eps <= k_cut)."""
    eps = np.asarray(eps, dtype=np.float64)
    yc = np.minimum(k_cut / np.maximum(eps, 1e-300), 1.0)
    if shape == CSBH:
        s = 4.0 / 3.0 * (-np.log(yc) - (1.0 - yc)) + 0.5 * (1.0 - yc * yc)
    else:
        s = -np.log(yc)
    return np.where(eps > k_cut, s, 0.0)


def sub_norm(eps, k_cut, shape):
    """S_sub(eps)/C_Z = int_0^{min(k_cut, eps)} phi(k/eps) dk  [J]."""
    eps = np.asarray(eps, dtype=np.float64)
    y = np.minimum(k_cut / np.maximum(eps, 1e-300), 1.0)
    if shape == CSBH:
        g = 4.0 / 3.0 * (y - 0.5 * y * y) + y ** 3 / 3.0
    else:
        g = y
    return eps * g


def cdf_x(x, eps, k_cut, shape):
    """F(x; eps): probability that an emitted photon (k >= k_cut) has
    ln(k/k_cut)/ln(eps/k_cut) <= x.  In y = k/eps: G(y)/G(1) with
    G(y) = int_{y_c}^{y} phi(t)/t dt and y = y_c^(1-x)."""
    yc = k_cut / eps
    y = yc ** (1.0 - np.asarray(x, dtype=np.float64))
    if shape == CSBH:
        g = 4.0 / 3.0 * (np.log(y / yc) - (y - yc)) + 0.5 * (y * y - yc * yc)
        g1 = 4.0 / 3.0 * (-np.log(yc) - (1.0 - yc)) + 0.5 * (1.0 - yc * yc)
    else:
        g = np.log(y / yc)
        g1 = -np.log(yc)
    return g / g1


class BremTable:
    """FP64 master table, built by bisection on the exact CDF."""

    def __init__(self, k_cut: float, emax: float, nT: int, nr: int, shape: int):
        self.k_cut, self.emax, self.nT, self.nr, self.shape = k_cut, emax, nT, nr, shape
        self.lnratio = math.log(emax / k_cut)
        j = np.arange(nT, dtype=np.float64)
        self.eps = k_cut * np.exp(self.lnratio * j / (nT - 1))
        self.r = np.arange(nr, dtype=np.float64) / (nr - 1)
        self.SIG = sigma_norm(self.eps, k_cut, shape)
        self.SUB = sub_norm(self.eps, k_cut, shape)
        X = np.empty((nT, nr))
        X[0, :] = self.r          # eps -> k_cut: phi ~ phi(1), ln k uniform
        for jj in range(1, nT):
            lo = np.zeros(nr)
            hi = np.ones(nr)
            for _ in range(64):   # bisection to below one ulp of [0, 1]
                mid = 0.5 * (lo + hi)
                below = cdf_x(mid, self.eps[jj], k_cut, shape) < self.r
                lo = np.where(below, mid, lo)
                hi = np.where(below, hi, mid)
            X[jj, :] = 0.5 * (lo + hi)
            X[jj, 0] = 0.0
            X[jj, -1] = 1.0
        self.X = X

    # --- lookups (linear in r, then linear in ln eps) ---------------------
    def _row(self, eps):
        s = (self.nT - 1) * np.log(np.maximum(eps, self.k_cut) / self.k_cut) / self.lnratio
        s = np.clip(s, 0.0, self.nT - 1)
        j = np.minimum(np.floor(s).astype(np.int64), self.nT - 2)
        return j, s - j

    def sigma(self, eps):
        """sigma(eps)/C_Z by table interpolation; 0 for eps <= k_cut."""
        eps = np.asarray(eps, dtype=np.float64)
        j, f = self._row(eps)
        v = self.SIG[j] + f * (self.SIG[j + 1] - self.SIG[j])
        return np.where(eps > self.k_cut, v, 0.0)

    def sub(self, eps):
        """S_sub(eps)/C_Z by table interpolation; eps itself below k_cut."""
        eps = np.asarray(eps, dtype=np.float64)
        j, f = self._row(eps)
        v = self.SUB[j] + f * (self.SUB[j + 1] - self.SUB[j])
        return np.where(eps > self.k_cut, v, eps)

    def sample_x(self, eps, r):
        eps = np.asarray(eps, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        j, f = self._row(eps)
        q = r * (self.nr - 1)
        i = np.minimum(np.floor(q).astype(np.int64), self.nr - 2)
        g = q - i
        x0 = self.X[j, i] + g * (self.X[j, i + 1] - self.X[j, i])
        x1 = self.X[j + 1, i] + g * (self.X[j + 1, i + 1] - self.X[j + 1, i])
        return x0 + f * (x1 - x0)

    def sample_k(self, eps, r):
        """Photon energy [J] for an electron of kinetic energy eps > k_cut."""
        x = self.sample_x(eps, r)
        return self.k_cut * np.exp(x * np.log(np.asarray(eps) / self.k_cut))
