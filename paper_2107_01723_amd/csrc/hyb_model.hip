// The paper's energy-partition model (Sec. III.B) on the GPU: at each point
// of an intensity-Z scan, the exponential injection is condensed into three
// macro-electrons and each is integrated through the continuous stopping
// powers of bremsstrahlung (eq. stop_brem), ionisation (eq. stop_ion),
// reflux (eq. stop_tnsa) and the resistive field (eq. stop_field).
//
// Four lanes per scan point: lanes 0-2 integrate the warm, emitting and
// escaping macro-electrons, lane 3 idles; their weighted losses are summed
// over the four lanes with shuffles in a fixed order.  The integrations are
// serial ODEs (fourth-order Runge-Kutta in u = ln(1 + eps / 1 keV)), so the
// kernel is FP64-ALU bound; a scan of a few thousand points fills the chip
// with a few thousand waves.
#include <hip/hip_runtime.h>
#include <math.h>

#include "hyb.h"
#include "hyb_internal.h"
#include "hyb_kernels.h"

namespace hyb {

namespace {

constexpr double kEpsS = 1e3 * kE;   // energy scale of the integration variable [J]

// constants of one scan point
struct ModelPoint {
  double k_brem;    // eq. stop_brem: k_brem * gamma
  double e_th;      // X-ray threshold
  double c_ion;     // eq. stop_ion prefactor times v^2: Z n_i e^4 / (4 pi eps0^2 m)
  double I_ex;      // mean excitation energy 11 eV Z
  double s_tnsa;    // eq. stop_tnsa
  double k_field;   // eq. stop_field numerator
  double tan_c, r_half;
};

// stopping powers [J/m] at kinetic energy eps and path x
struct Stop { double brem, thr, ion, tnsa, field; };

__device__ __forceinline__ Stop stopping(const ModelPoint& p, double eps, double x) {
  Stop s;
  const double g = 1.0 + eps / kMec2;
  s.brem = p.k_brem * g;
  s.thr = eps > p.e_th ? p.k_brem * (1.0 + (eps - p.e_th) / kMec2) : 0.0;
  s.ion = 0.0;
  if (eps > 0.0) {
    const double v2 = kC * kC * (1.0 - 1.0 / (g * g));
    const double L = log(eps / p.I_ex) + 0.5 * log(g + 1.0) + 0.909 / (g * g) - 0.818 / g - 0.246;
    const double S = p.c_ion / v2 * L;
    s.ion = S > 0.0 ? S : 0.0;
  }
  s.tnsa = p.s_tnsa;
  const double d = x * p.tan_c + p.r_half;
  s.field = p.k_field / (d * d);
  return s;
}

// d(x, E_brem, E_thr, E_ion, E_tnsa, E_field) / d(-u) per electron
__device__ __forceinline__ void rhs(const ModelPoint& p, double u, const double (&y)[6], double (&k)[6]) {
  const double eps = kEpsS * expm1(u);
  const Stop s = stopping(p, eps, y[0]);
  const double de = kEpsS * exp(u) / (s.brem + s.ion + s.tnsa + s.field);
  k[0] = de;
  k[1] = de * s.brem;
  k[2] = de * s.thr;
  k[3] = de * s.ion;
  k[4] = de * s.tnsa;
  k[5] = de * s.field;
}

__global__ __launch_bounds__(64) void k_model(hyb_model m, const double* __restrict__ I0,
                                              const double* __restrict__ Zs, long long n,
                                              double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pt = t >> 2;
  const int q = (int)(t & 3);   // 0 warm, 1 emitting, 2 escaping, 3 idle
  const bool live = pt < n;
  const double I = live ? I0[pt] : 1.0, Z = live ? Zs[pt] : 1.0;
  // point constants
  const double a0 = 8.5e-6 * sqrt(I * m.wavelength * m.wavelength);
  const double T = a0 * kMec2 * m.sqrt_fg_mean;
  const double N = I * m.fg_mean * (kPi * m.r_fwhm * m.r_fwhm / 4.0) *
                   (m.t_fwhm * sqrt(log(10.0) / log(2.0))) * m.eta_l2e / T;
  ModelPoint p;
  p.k_brem = kE * kE * kE * kE * kE * kE / (12.0 * kPi * kPi * kPi * kEps0 * kEps0 * kEps0 * kMe * kC * kC * kC * kHbar) *
             m.n_i * Z * Z * log(5.6 * kPi * kEps0 * kHbar * kC / (pow(Z, 1.0 / 3.0) * kE * kE));
  p.e_th = m.e_th;
  p.c_ion = Z * m.n_i * kE * kE * kE * kE / (4.0 * kPi * kEps0 * kEps0 * kMe);
  p.I_ex = 11.0 * kE * Z;
  p.s_tnsa = 3.0 * m.kappa_tnsa * a0 * kMec2 / (m.Lx + m.Ly + m.Lz);
  p.k_field = kE * kE * m.eta_mean * I * m.fg_mean * (0.5 * m.r_fwhm) * (0.5 * m.r_fwhm) * m.eta_l2e / T;
  p.tan_c = tan(m.theta_c);
  p.r_half = 0.5 * m.r_fwhm;
  // this lane's bin of the exponential: [lo, hi); e1 = min(e_th, e_esc)
  const double e_esc = m.kappa_esc * a0 * kMec2;
  const double e1 = fmin(m.e_th, e_esc);
  const double lo = q == 0 ? 0.0 : (q == 1 ? e1 : e_esc);
  const double ex_lo = exp(-lo / T);
  const double cn_lo = 1.0 - ex_lo, ce_lo = T - (lo + T) * ex_lo;
  double cn_hi = 1.0, ce_hi = T;   // the open top bin
  if (q < 2) {
    const double hi = q == 0 ? e1 : e_esc;
    const double ex_hi = exp(-hi / T);
    cn_hi = 1.0 - ex_hi;
    ce_hi = T - (hi + T) * ex_hi;
  }
  const double W = (live && q < 3) ? N * (cn_hi - cn_lo) : 0.0;
  const double E = (live && q < 3) ? N * (ce_hi - ce_lo) : 0.0;
  double loss[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double left = 0.0;
  if (W > 0.0) {
    const double eps0 = E / W;
    const double x_stop = q == 2 ? m.Lx : INFINITY;
    const double u0 = log1p(eps0 / kEpsS);
    const double h = u0 / m.nsteps;
    double y[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double u = u0;
    for (int k = 0; k < m.nsteps; ++k) {
      // u runs from u0 down to exactly 0
      const double um = u0 * ((m.nsteps - k - 0.5) / m.nsteps);
      const double u1 = u0 * ((m.nsteps - k - 1.0) / m.nsteps);
      double k1[6], k2[6], k3[6], k4[6], yt[6];
      rhs(p, u, y, k1);
#pragma unroll
      for (int j = 0; j < 6; ++j) yt[j] = y[j] + 0.5 * h * k1[j];
      rhs(p, um, yt, k2);
#pragma unroll
      for (int j = 0; j < 6; ++j) yt[j] = y[j] + 0.5 * h * k2[j];
      rhs(p, um, yt, k3);
#pragma unroll
      for (int j = 0; j < 6; ++j) yt[j] = y[j] + h * k3[j];
      rhs(p, u1, yt, k4);
      double y1[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) y1[j] = y[j] + h / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
      if (y1[0] >= x_stop) {
        // the path reaches x_stop inside this step: interpolate, and what
        // has not been lost escapes (photon_thr is part of brem)
        const double s = (x_stop - y[0]) / (y1[0] - y[0]);
#pragma unroll
        for (int j = 0; j < 6; ++j) y[j] = y[j] + s * (y1[j] - y[j]);
        left = eps0 - (y[1] + y[3] + y[4] + y[5]);
        break;
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) y[j] = y1[j];
      u = u1;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) loss[j] = W * y[j + 1];
    left *= W;
  }
  // sums over the point's four lanes, fixed order
  double v[7] = {loss[0], loss[1], loss[2], loss[3], loss[4], left, E};
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    v[j] += __shfl_xor(v[j], 1, 64);
    v[j] += __shfl_xor(v[j], 2, 64);
  }
  if (live && q == 0) {
    const double inv = 1.0 / v[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) out[6 * pt + j] = v[j] * inv;
  }
}

}  // namespace

void launch_model(const hyb_model& m, const double* I0, const double* Z, long long n, double* out,
                  hipStream_t s) {
  const long long threads = 4 * n;
  const long long blocks = (threads + 63) / 64;
  hipLaunchKernelGGL(k_model, dim3((unsigned)blocks), dim3(64), 0, s, m, I0, Z, n, out);
}

}  // namespace hyb
