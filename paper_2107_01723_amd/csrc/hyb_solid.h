// Background solid of the hybrid model (App. A of the paper), FP64, callable
// on host (initial state, stability scan) and device (per-cell update).
// Temperatures in kelvin, SI otherwise.
#pragma once

#include <math.h>

#include "hyb_internal.h"

namespace hyb {

// Ionisation state: More's Thomas-Fermi fit (the paper's "More Table IV
// algorithm"), temperature in eV and density in g/cm^3 inside.
__host__ __device__ inline double zstar(double Z, double A, double rho, double Te) {
  const double alpha = 14.3139, beta = 0.6624;
  const double a1 = 0.003323, a2 = 0.971832, a3 = 9.26148e-5, a4 = 3.10165;
  const double b0 = -1.7630, b1 = 1.43175, b2 = 0.31546;
  const double c1 = -0.366667, c2 = 0.983333;
  const double Tev = Te * kKb / kE;
  const double R = rho * 1e-3 / (A * Z);
  const double T0 = Tev / pow(Z, 4.0 / 3.0);
  const double Tf = T0 / (1.0 + T0);
  const double Ac = a1 * pow(T0, a2) + a3 * pow(T0, a4);
  const double Bc = -exp(b0 + b1 * Tf + b2 * pow(Tf, 7.0));
  const double Cc = c1 * Tf + c2;
  const double Q1 = Ac * pow(R, Bc);
  const double Q = pow(pow(R, Cc) + pow(Q1, Cc), 1.0 / Cc);
  const double x = alpha * pow(Q, beta);
  return Z * x / (1.0 + x + sqrt(1.0 + 2.0 * x));
}

// Coulomb logarithm (Lee-More style bounds): max(2, ln(1 + (bmax/bmin)^2)/2)
// with bmax = max(Debye length, ion-sphere radius) and bmin = max(classical
// distance of closest approach, electron de Broglie length), electron
// temperature replaced by sqrt(Te^2 + TF^2).
__host__ __device__ inline double coulomb_log(double Te, double Ti, double Zs, double n_i) {
  const double ne = Zs * n_i;
  const double TF = kHbar * kHbar * pow(3.0 * kPi * kPi * ne, 2.0 / 3.0) / (2.0 * kMe * kKb);
  const double Teff = sqrt(Te * Te + TF * TF);
  const double inv_ld2 = kE * kE * ne / (kEps0 * kKb * Teff) + Zs * Zs * kE * kE * n_i / (kEps0 * kKb * Ti);
  const double lam_d = 1.0 / sqrt(inv_ld2);
  const double R0 = cbrt(3.0 / (4.0 * kPi * n_i));
  const double bmax = fmax(lam_d, R0);
  const double bmin = fmax(Zs * kE * kE / (12.0 * kPi * kEps0 * kKb * Teff),
                           kHbar / (2.0 * sqrt(3.0 * kMe * kKb * Teff)));
  const double r = bmax / bmin;
  return fmax(2.0, 0.5 * log(1.0 + r * r));
}

// Reduced Lee-More resistivity eq. (LeeMoreGeneral) times lambda2, with
// tau A = max(hot, cold) limits of App. A.
__host__ __device__ inline double resistivity(double Te, double Ti, double Z, double A, double rho,
                                              double n_i, double lambda1, double lambda2) {
  const double Zs = zstar(Z, A, rho, Te);
  const double lnL = coulomb_log(Te, Ti, Zs, n_i);
  const double kT = kKb * Te;
  const double tau_hot = 128.0 * kPi * kEps0 * kEps0 / (3.0 * kE * kE * kE * kE) *
                         sqrt(kMe / (2.0 * kPi)) * kT * sqrt(kT) / (Zs * Zs * n_i * lnL);
  const double R0 = cbrt(3.0 / (4.0 * kPi * n_i));
  const double tau_cold = lambda1 * R0 / sqrt(3.0 * kT / kMe);
  return lambda2 * kMe / (Zs * n_i * kE * kE * fmax(tau_hot, tau_cold));
}

// Heat capacity per electron in units of kB, App. A.
__host__ __device__ inline double heat_capacity(double Te, double Z) {
  const double Tp = kKb * Te / kE / pow(Z, 4.0 / 3.0);
  return 0.3 + 1.2 * Tp * (2.2 + Tp) / ((1.1 + Tp) * (1.1 + Tp));
}

// One cell: Ohmic + collisional heating eq. (Te_rise), exact electron-ion
// exchange with rates frozen after heating, new resistivity.
__host__ __device__ inline void heat_cell(double& Te, double& Ti, double& eta, double j2, double ion_heat_J,
                                          double dt, double dV, double Z, double A, double rho, double n_i,
                                          double m_i, double lambda1, double lambda2, bool fixed_eta) {
  const double rho_eps = eta * j2 * dt + ion_heat_J / dV;
  const double C = heat_capacity(Te, Z);
  const double Te1 = Te + rho_eps / (Z * n_i * C * kKb);
  const double Zs1 = zstar(Z, A, rho, Te1);
  const double lnL1 = coulomb_log(Te1, Ti, Zs1, n_i);
  const double denom = Te1 * m_i + Ti * kMe;
  const double inv_tc = 2.0 / (3.0 * pow(2.0 * kPi * kKb, 1.5)) * sqrt(kMe * m_i) * lnL1 /
                        (kEps0 * kEps0 * denom * sqrt(denom));
  const double e4 = kE * kE * kE * kE;
  const double a = Zs1 * Zs1 * e4 * n_i * inv_tc;
  const double b = Zs1 * Zs1 * Zs1 * e4 * n_i * inv_tc;
  const double s = a + b;
  const double M = (b * Te1 + a * Ti) / s;
  const double D = (Te1 - Ti) * exp(-s * dt);
  const double Te2 = M + a / s * D;
  const double Ti2 = M - b / s * D;
  Te = Te2;
  Ti = Ti2;
  if (!fixed_eta) eta = resistivity(Te2, Ti2, Z, A, rho, n_i, lambda1, lambda2);
}

}  // namespace hyb
