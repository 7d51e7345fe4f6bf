// Background solid of the hybrid model (App. A of the paper), FP64, callable
// on host (initial state, stability scan) and device (per-cell update).
// Temperatures in kelvin, SI otherwise.  Powers with run-constant bases or
// exponents are taken through the constants of Solid and exp/log pairs.
#pragma once

#include <math.h>

#include "hyb_internal.h"

namespace hyb {

// Natural logarithm of a positive, finite x, within a few units in the last
// place: x = m 2^e with m in [sqrt(1/2), sqrt(2)), and ln m = 2 atanh(s),
// s = (m - 1) / (m + 1), |s| < 0.172, by its Taylor series
// 2 (s + s^3/3 + ... + s^23/23) (the next term is below 2^-60 of 2s);
// e ln 2 in two parts, the first exact for any exponent.  The per-cell
// update is bound by FP64 issue, and this takes a third of the
// instructions of the correctly rounded library logarithm.
__host__ __device__ inline double ln_pos(double x) {
  const double kLn2Hi = 0x1.62e42ffp-1, kLn2Lo = -0x1.718432a1b0e26p-35;
  int e;
  double m = frexp(x, &e);                     // [0.5, 1)
  if (m < 0x1.6a09e667f3bcdp-1) { m += m; --e; }   // [sqrt(1/2), sqrt(2))
  const double f = m - 1.0;                    // exact
  const double s = f / (m + 1.0), z = s * s;
  double p = 1.0 / 23.0;
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = s + s, de = (double)e;
  return fma(de, kLn2Hi, s2 + fma(s2 * z, p, de * kLn2Lo));
}

__host__ __device__ inline Solid make_solid(double Z, double A, double rho, double n_i, double lambda1,
                                            double lambda2) {
  Solid s;
  s.Z = Z; s.A = A; s.rho = rho; s.n_i = n_i; s.m_i = A * kAmu;
  s.lambda1 = lambda1; s.lambda2 = lambda2;
  s.z43 = pow(Z, 4.0 / 3.0);
  s.lnR = log(rho * 1e-3 / (A * Z));
  s.tf_c = kHbar * kHbar * pow(3.0 * kPi * kPi, 2.0 / 3.0) / (2.0 * kMe * kKb);
  s.r0 = cbrt(3.0 / (4.0 * kPi * n_i));
  s.th_c = 128.0 * kPi * kEps0 * kEps0 / (3.0 * kE * kE * kE * kE) * sqrt(kMe / (2.0 * kPi));
  s.tc_c = 2.0 / (3.0 * pow(2.0 * kPi * kKb, 1.5)) * sqrt(kMe * s.m_i) / (kEps0 * kEps0);
  const double a_bohr = 4.0 * kPi * kEps0 * kHbar * kHbar / (kMe * kE * kE);
  s.a_s = 1.4 * a_bohr / cbrt(Z);
  s.ln_as = log(s.a_s * kMe * kC / kHbar);
  s.t_ev = kKb / kE / s.z43;
  s.ld_e = kE * kE / (kEps0 * kKb);
  s.ld_i = kE * kE * n_i / (kEps0 * kKb);
  const double bc = kE * kE / (12.0 * kPi * kEps0 * kKb);
  s.bc2 = bc * bc;
  s.bq2 = kHbar * kHbar / (12.0 * kMe * kKb);
  s.r02 = s.r0 * s.r0;
  s.inv_znk = 1.0 / (Z * n_i * kKb);
  s.tcold = lambda1 * s.r0 * sqrt(kMe / 3.0);
  s.eta_c = lambda2 * kMe / (n_i * kE * kE);
  return s;
}

// Ionisation state: More's Thomas-Fermi fit (the paper's "More Table IV
// algorithm"), temperature in eV and density in g/cm^3 inside.
__host__ __device__ inline double zstar(const Solid& s, double Te) {
  const double alpha = 14.3139, beta = 0.6624;
  const double a1 = 0.003323, a2 = 0.971832, a3 = 9.26148e-5, a4 = 3.10165;
  const double b0 = -1.7630, b1 = 1.43175, b2 = 0.31546;
  const double c1 = -0.366667, c2 = 0.983333;
  const double kLnA1 = -5.706887289609679;   // ln a1
  const double T0 = Te * s.t_ev;
  const double Tf = T0 / (1.0 + T0);
  const double lnT0 = ln_pos(T0);
  // ln A = ln(a1 T0^a2 + a3 T0^a4) = ln a1 + a2 ln T0 + ln(1 + (a3/a1) T0^(a4-a2))
  const double lnA = kLnA1 + a2 * lnT0 + ln_pos(1.0 + (a3 / a1) * exp((a4 - a2) * lnT0));
  const double Tf2 = Tf * Tf, Tf7 = Tf2 * Tf2 * Tf2 * Tf;
  const double Bc = -exp(b0 + b1 * Tf + b2 * Tf7);
  const double Cc = c1 * Tf + c2;                                    // > 0.6 for Tf in [0, 1]
  const double lnQ1 = lnA + Bc * s.lnR;                              // Q1 = A R^Bc
  // Q = (R^C + Q1^C)^(1/C): ln Q = max + ln(1 + e^(-C |ln Q1 - ln R|)) / C
  // (the second term is taken to an absolute, not relative, accuracy)
  const double dl = lnQ1 - s.lnR;
  const double lnQ = (dl > 0.0 ? lnQ1 : s.lnR) + ln_pos(1.0 + exp(-Cc * fabs(dl))) / Cc;
  const double x = alpha * exp(beta * lnQ);
  return s.Z * x / (1.0 + x + sqrt(1.0 + 2.0 * x));
}

// Coulomb logarithm (Lee-More style bounds): max(2, ln(1 + (bmax/bmin)^2)/2)
// with bmax = max(Debye length, ion-sphere radius) and bmin = max(classical
// distance of closest approach, electron de Broglie length), electron
// temperature replaced by sqrt(Te^2 + TF^2).
__host__ __device__ inline double coulomb_log(const Solid& s, double Te, double Ti, double Zs) {
  const double ne = Zs * s.n_i;
  const double c = cbrt(ne);
  const double TF = s.tf_c * c * c;
  const double rT = 1.0 / sqrt(Te * Te + TF * TF);   // 1 / Teff
  const double inv_ld2 = s.ld_e * ne * rT + s.ld_i * Zs * Zs / Ti;
  const double bmax2 = fmax(1.0 / inv_ld2, s.r02);
  const double bmin2 = fmax(s.bc2 * Zs * Zs * rT * rT, s.bq2 * rT);
  return fmax(2.0, 0.5 * ln_pos(1.0 + bmax2 / bmin2));
}

// Bremsstrahlung enhancement by the ionised background, eq. (F_sigma):
// 1 + ln|lambda_D / a_s| / ln(a_s m_e c / hbar) (Z*/Z)^2, lambda_D the Debye
// length of the background ions (the printed m_e c^2 read as m_e c, which
// makes the denominator the dimensionless complete-screening logarithm).
__host__ __device__ inline double f_sigma(const Solid& s, double Ti, double Zs) {
  const double lam = sqrt(kEps0 * kKb * Ti / (Zs * Zs * kE * kE * s.n_i));
  const double q = Zs / s.Z;
  return 1.0 + log(fabs(lam / s.a_s)) / s.ln_as * q * q;
}

// Reduced Lee-More resistivity eq. (LeeMoreGeneral) times lambda2, with
// tau = max(hot, cold) limits of App. A; Zs = Z*(Te).
__host__ __device__ inline double resistivity_z(const Solid& s, double Te, double Ti, double Zs) {
  const double lnL = coulomb_log(s, Te, Ti, Zs);
  const double kT = kKb * Te, skT = sqrt(kT);
  const double tau_hot = s.th_c * kT * skT / (Zs * Zs * s.n_i * lnL);
  const double tau_cold = s.tcold / skT;             // lambda1 r0 / sqrt(3 k_B Te / m_e)
  return s.eta_c / (Zs * fmax(tau_hot, tau_cold));
}

__host__ __device__ inline double resistivity(const Solid& s, double Te, double Ti) {
  return resistivity_z(s, Te, Ti, zstar(s, Te));
}

// Heat capacity per electron in units of kB, App. A.
__host__ __device__ inline double heat_capacity(const Solid& s, double Te) {
  const double Tp = Te * s.t_ev;
  return 0.3 + 1.2 * Tp * (2.2 + Tp) / ((1.1 + Tp) * (1.1 + Tp));
}

// One cell: Ohmic + collisional heating eq. (Te_rise), exact electron-ion
// exchange with rates frozen after heating, new resistivity and, if want_fs,
// the new eq. (F_sigma) factor in fs.
__host__ __device__ inline void heat_cell(const Solid& s, double& Te, double& Ti, double& eta, double j2,
                                          double ion_heat_J, double dt, double dV, bool fixed_eta,
                                          bool want_fs, double& fs) {
  const double rho_eps = eta * j2 * dt + ion_heat_J / dV;
  const double C = heat_capacity(s, Te);
  const double Te1 = Te + rho_eps * s.inv_znk / C;
  const double Zs1 = zstar(s, Te1);
  const double lnL1 = coulomb_log(s, Te1, Ti, Zs1);
  const double denom = Te1 * s.m_i + Ti * kMe;
  const double inv_tc = s.tc_c * lnL1 / (denom * sqrt(denom));
  const double e4 = kE * kE * kE * kE;
  const double a = Zs1 * Zs1 * e4 * s.n_i * inv_tc;
  const double b = Zs1 * Zs1 * Zs1 * e4 * s.n_i * inv_tc;
  const double sum = a + b, rs = 1.0 / sum;
  const double M = (b * Te1 + a * Ti) * rs;
  const double D = (Te1 - Ti) * exp(-sum * dt);
  const double Te2 = M + a * rs * D;
  const double Ti2 = M - b * rs * D;
  Te = Te2;
  Ti = Ti2;
  if (fixed_eta && !want_fs) return;
  const double Zs2 = zstar(s, Te2);
  if (!fixed_eta) eta = resistivity_z(s, Te2, Ti2, Zs2);
  if (want_fs) fs = f_sigma(s, Ti2, Zs2);
}

// Compound resistivity: sum(x Z* eta_el) / sum(x Z*), each element's
// Lee-More resistivity as if it filled the cell at the total ion density
// (the free electrons' collision rates add over the ion species).
__host__ __device__ inline double resistivity_mix(const Mix& m, double Te, double Ti) {
  if (m.n == 1) return resistivity(m.el[0], Te, Ti);
  double num = 0.0, den = 0.0;
  for (int k = 0; k < m.n; ++k) {
    const double Zs = zstar(m.el[k], Te);
    num += m.x[k] * Zs * resistivity_z(m.el[k], Te, Ti, Zs);
    den += m.x[k] * Zs;
  }
  return num / den;
}

// One cell of a compound (App. A): heating with n_e summed over the
// elements and 1/C averaged with weights Z n; electron-ion exchange with the
// elements' rates added by ion share, the ions' rate scaled by the mean Z*
// (energy conservation between free electrons and ions); the compound
// resistivity.  One element: heat_cell.
__host__ __device__ inline void heat_cell_mix(const Mix& m, double& Te, double& Ti, double& eta, double j2,
                                              double ion_heat_J, double dt, double dV, bool fixed_eta,
                                              bool want_fs, double& fs) {
  if (m.n == 1) {
    heat_cell(m.el[0], Te, Ti, eta, j2, ion_heat_J, dt, dV, fixed_eta, want_fs, fs);
    return;
  }
  const double rho_eps = eta * j2 * dt + ion_heat_J / dV;
  double inv_c = 0.0;
  for (int k = 0; k < m.n; ++k) inv_c += m.w[k] / heat_capacity(m.el[k], Te);
  const double Te1 = Te + rho_eps * inv_c / (m.ne * kKb);
  const double e4 = kE * kE * kE * kE;
  double a = 0.0, zbar = 0.0;
  for (int k = 0; k < m.n; ++k) {
    const Solid& s = m.el[k];
    const double Zs = zstar(s, Te1);
    const double lnL = coulomb_log(s, Te1, Ti, Zs);
    const double denom = Te1 * s.m_i + Ti * kMe;
    const double inv_tc = s.tc_c * lnL / (denom * sqrt(denom));
    a += m.x[k] * Zs * Zs * e4 * s.n_i * inv_tc;
    zbar += m.x[k] * Zs;
  }
  const double b = a * zbar;
  const double sum = a + b;
  const double M = (b * Te1 + a * Ti) / sum;
  const double D = (Te1 - Ti) * exp(-sum * dt);
  Te = M + a / sum * D;
  Ti = M - b / sum * D;
  if (!fixed_eta) eta = resistivity_mix(m, Te, Ti);
}

}  // namespace hyb
