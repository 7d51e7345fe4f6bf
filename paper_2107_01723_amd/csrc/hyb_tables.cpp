// Host builder of the bremsstrahlung cross-section tables (FP64 master).
//
// The optical-depth method (App. B of the paper) needs the total
// cross-section sigma(eps) of photon emission above k_cut and the photon
// energy distribution at each electron energy.  The spectral shape is
//   k dsigma/dk = C_Z phi(k/eps),  0 < k <= eps,
//   CSBH: phi(y) = 4/3 (1 - y) + y^2,   FLAT: phi(y) = 1,
// with C_Z the prefactor of eq. (stop_brem); both shapes integrate to one
// over y, so the total radiative stopping reproduces eq. (stop_brem).
// Rows are log-spaced electron energies k_cut .. emax; columns the variate
// r in [0, 1]; X holds x = ln(k/k_cut)/ln(eps/k_cut) with F(x; eps) = r,
// found by bisection on the closed-form CDF.
#include <math.h>

#include <vector>

#include "hyb_tables.h"

namespace hyb {

static double sigma_norm(double eps, double kcut, int shape) {
  if (!(eps > kcut)) return 0.0;
  const double yc = kcut / eps;
  if (shape == 0) return 4.0 / 3.0 * (-log(yc) - (1.0 - yc)) + 0.5 * (1.0 - yc * yc);
  return -log(yc);
}

static double sub_norm(double eps, double kcut, int shape) {
  double y = kcut / eps;
  if (y > 1.0) y = 1.0;
  const double g = shape == 0 ? 4.0 / 3.0 * (y - 0.5 * y * y) + y * y * y / 3.0 : y;
  return eps * g;
}

// F(x; eps): probability that an emitted photon has ln(k/kcut)/ln(eps/kcut) <= x
static double cdf_x(double x, double eps, double kcut, int shape) {
  const double yc = kcut / eps;
  const double y = pow(yc, 1.0 - x);
  double g, g1;
  if (shape == 0) {
    g = 4.0 / 3.0 * (log(y / yc) - (y - yc)) + 0.5 * (y * y - yc * yc);
    g1 = 4.0 / 3.0 * (-log(yc) - (1.0 - yc)) + 0.5 * (1.0 - yc * yc);
  } else {
    g = log(y / yc);
    g1 = -log(yc);
  }
  return g / g1;
}

void build_brem_table(double kcut, double emax, int nT, int nr, int shape, std::vector<double>& X,
                      std::vector<double>& SIG, std::vector<double>& SUB) {
  X.assign((size_t)nT * nr, 0.0);
  SIG.assign(nT, 0.0);
  SUB.assign(nT, 0.0);
  const double lnratio = log(emax / kcut);
  for (int j = 0; j < nT; ++j) {
    const double eps = kcut * exp(lnratio * j / (nT - 1));
    SIG[j] = sigma_norm(eps, kcut, shape);
    SUB[j] = sub_norm(eps, kcut, shape);
    for (int i = 0; i < nr; ++i) {
      const double r = (double)i / (nr - 1);
      double x;
      if (j == 0) {
        x = r;   // eps -> kcut: ln k uniform
      } else if (i == 0) {
        x = 0.0;
      } else if (i == nr - 1) {
        x = 1.0;
      } else {
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 64; ++it) {
          const double mid = 0.5 * (lo + hi);
          if (cdf_x(mid, eps, kcut, shape) < r) lo = mid;
          else hi = mid;
        }
        x = 0.5 * (lo + hi);
      }
      X[(size_t)j * nr + i] = x;
    }
  }
}

}  // namespace hyb
