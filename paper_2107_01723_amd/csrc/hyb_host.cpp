// Host runtime of the MI355X hybrid-PIC library: the C ABI of include/hyb.h.
//
// A run owns one device allocation carved into fields, cell arrays,
// double-buffered structure-of-arrays particles, tables and accumulators,
// plus a device-resident run descriptor.  Steps are enqueued on the
// caller's stream as batched kernels (a batch of one here, many in the
// serving engine), optionally captured once as a HIP graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hyb.h"
#include "hyb_internal.h"
#include "hyb_kernels.h"
#include "hyb_solid.h"
#include "hyb_tables.h"

using namespace hyb;

namespace {

constexpr int kRedBlocks = 1024;   // partial-sum slots of the kinetic reduction

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// words per copy of the photon-tally accumulators (rounded to 128 bytes)
size_t hist_stride(const hyb_config& c) {
  return align_up(2 * (size_t)c.tally_nE * c.tally_ntheta + 4, 16);
}

// Sizes of everything a run keeps in device memory.
struct Layout {
  size_t off_E[3], off_B[3], off_J[3], off_Te, off_Ti, off_eta[2], off_heat, off_fsig;
  size_t off_Jacc[3], off_heat_acc, off_stamp, off_dirty, off_pj, off_ph;
  size_t off_part[2][11];
  size_t off_sp_cell, off_sp_pid, off_sp_f[7], off_sp_cnt, off_sp_start, off_sp_blk, off_sp_grp, off_sp_gpid;
  size_t off_tabX, off_tabSIG, off_tabSUB;
  size_t off_acc_led, off_acc_hist, off_events, off_tot_led, off_tot_led_c, off_tot_hist, off_tot_hist_c;
  size_t off_series, off_ctr, off_src, off_env, off_tile_cnt, off_tile_start, off_scan_blk,
         off_chunk_home, off_chunk_base, off_far, off_red, off_desc;
  size_t total;
};

Layout make_layout(const hyb_config& c) {
  Layout L{};
  const size_t ts = c.precision == HYB_FP64 ? 8 : 4;
  const size_t nodes = (size_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
  const size_t cells = (size_t)c.nx * c.ny * c.nz;
  const size_t cap = (size_t)c.max_particles;
  const bool delta = (c.physics & HYB_PHYS_DELTA) != 0;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  for (int d = 0; d < 3; ++d) L.off_E[d] = take(nodes * ts);
  for (int d = 0; d < 3; ++d) L.off_B[d] = take(nodes * ts);
  for (int d = 0; d < 3; ++d) L.off_J[d] = take(nodes * 8);
  L.off_Te = take(cells * 8);
  L.off_Ti = take(cells * 8);
  for (int k = 0; k < 2; ++k) L.off_eta[k] = take(cells * 8);
  L.off_heat = take(cells * 8);
  L.off_fsig = take(cells * ts);
  // the particle kernel's accumulators and per-tile partials, summed into
  // J and the heat by the gather
  const size_t ntl = (size_t)((c.nx + kTile - 1) / kTile) * ((c.ny + kTile - 1) / kTile) *
                     ((c.nz + kTile - 1) / kTile);
  for (int d = 0; d < 3; ++d) L.off_Jacc[d] = take(nodes * 8);
  L.off_heat_acc = take(cells * 8);
  L.off_stamp = take(ntl * 4);
  L.off_dirty = take(ntl * 4);
  L.off_pj = take(ntl * 3 * kPjWords * ts);
  L.off_ph = take(ntl * kTile * kTile * kTile * 8);
  for (int b = 0; b < 2; ++b) {
    // one record per electron: cell, id, then ox oy oz ux uy uz wn tau
    const size_t rec = 8 + 8 * ts;
    L.off_part[b][0] = take(cap * rec);                     // cell
    L.off_part[b][9] = L.off_part[b][0] + 4;                // id
    for (int f = 1; f < 9; ++f) L.off_part[b][f] = L.off_part[b][0] + 8 + (f - 1) * ts;
    L.off_part[b][10] = take(delta ? cap * ts : 0);         // delta-ray depth (own array)
  }
  const size_t tabn = (size_t)c.table_nT * c.table_nr;
  L.off_tabX = take(tabn * ts);
  L.off_tabSIG = take((size_t)c.table_nT * ts);
  L.off_tabSUB = take((size_t)c.table_nT * ts);
  const size_t nh = 2 * (size_t)c.tally_nE * c.tally_ntheta + 4;
  L.off_acc_led = take(16 * 8);
  L.off_acc_hist = take(hist_stride(c) * kHistCopies * 8);
  L.off_events = take(16 * 8);
  L.off_tot_led = take(16 * 8);
  L.off_tot_led_c = take(16 * 8);
  L.off_tot_hist = take(nh * 8);
  L.off_tot_hist_c = take(nh * 8);
  L.off_series = take((size_t)std::max(1, c.series_len) * 8);
  L.off_ctr = take(sizeof(Counters));
  L.off_src = take(sizeof(SourceDesc) * kMaxSources);
  L.off_env = take((size_t)kMaxSources * c.ny * c.nz * 4);
  const size_t ntiles = (size_t)((c.nx + kTile - 1) / kTile) * ((c.ny + kTile - 1) / kTile) *
                        ((c.nz + kTile - 1) / kTile);
  L.off_tile_cnt = take(ntiles * 4);
  L.off_tile_start = take(ntiles * 4);
  L.off_scan_blk = take(((ntiles + kScanTile - 1) / kScanTile) * 4);
  const size_t nchunks = (cap + kChunk - 1) / kChunk;
  L.off_chunk_home = take(nchunks * 4);
  L.off_chunk_base = take(nchunks * kNbN * 4);
  L.off_far = take(cap * 4);
  // delta-ray records: one per particle slot at most
  const size_t spc = delta ? cap : 0;
  L.off_sp_cell = take(spc * 4);
  L.off_sp_pid = take(spc * 4);
  for (int f = 0; f < 7; ++f) L.off_sp_f[f] = take(spc * ts);
  L.off_sp_cnt = take(delta ? ntiles * 4 : 0);
  L.off_sp_start = take(delta ? ntiles * 4 : 0);
  L.off_sp_blk = take(delta ? ((ntiles + kScanTile - 1) / kScanTile) * 4 : 0);
  L.off_sp_grp = take(spc * 4);
  L.off_sp_gpid = take(spc * 4);
  L.off_red = take(2 * kRedBlocks * 8);
  L.off_desc = take(sizeof(RunDesc));
  L.total = o;
  return L;
}

double cz_of(double Z) {
  const double alpha = kE * kE / (4.0 * kPi * kEps0 * kHbar * kC);
  const double re = kE * kE / (4.0 * kPi * kEps0 * kMec2);
  return 16.0 / 3.0 * alpha * re * re * Z * Z * log(1.4 / alpha * pow(Z, -1.0 / 3.0));
}

int clampi(long long v, int lo, int hi) { return (int)std::max<long long>(lo, std::min<long long>(hi, v)); }

}  // namespace

struct hyb_engine;

struct hyb_run {
  hyb_config cfg{};
  hyb_device dev{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  hipStream_t side = nullptr, side2 = nullptr;   // field sub-cycles, heating beside the sort
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  hyb_engine* eng = nullptr;
  int slot = -1;
  void* base = nullptr;
  size_t bytes = 0;
  Layout lay{};
  RunDesc h{};
  RunDesc* d_desc = nullptr;
  std::vector<SourceDesc> srcs;
  std::vector<double> tabX, tabSIG, tabSUB;
  // single-run launch plans
  LaunchSet L;
  BlockMap* d_maps = nullptr;
  size_t maps_bytes = 0;
  int64_t next_id = 0, scheduled = 0;
  double w_ref = 0.0;
  bool w_locked = false;
  int64_t host_step = 0;
  int32_t nsteps_engine = 0;
  std::string err;
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  double t_ms = 0.0;
  int64_t t_n = 0;
  int64_t solid_cells = 0;
};

static thread_local std::string g_err;   // last error of a call that has no run handle

static hyb_status fail(hyb_run* r, hyb_status s, const std::string& msg) {
  if (r) r->err = msg;
  g_err = msg;
  return s;
}

#define HIPCHK(r, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((r), HYB_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// configuration
// ---------------------------------------------------------------------------
static std::string validate(const hyb_config& c) {
  if (c.nx < 2 || c.ny < 2 || c.nz < 2) return "nx, ny, nz must be >= 2";
  if (c.nx >= 2048 || c.ny >= 1024 || c.nz >= 2048) return "grid too large for the packed cell index";
  const double nodes = (double)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
  if (nodes >= 2147483647.0) return "grid has too many nodes";
  if (!(c.dx > 0) || !(c.dt > 0)) return "dx and dt must be positive";
  if (c.precision != HYB_FP64 && c.precision != HYB_FP32_MIXED) return "precision must be HYB_FP64 or HYB_FP32_MIXED";
  if (!(c.Z >= 1) || !(c.A > 0) || !(c.rho > 0)) return "bad solid (Z, A, rho)";
  const double lo = c.x_lo / c.dx, hi = c.x_hi / c.dx;
  if (fabs(lo - llround(lo)) > 1e-6 || fabs(hi - llround(hi)) > 1e-6) return "slab faces must lie on cell faces";
  if (llround(lo) < 0 || llround(hi) > c.nx || llround(lo) >= llround(hi)) return "slab outside the grid";
  if (!(c.T0 > 0)) return "T0 must be positive";
  if (!(c.lambda1 > 0) || !(c.lambda2 > 0)) return "lambda1, lambda2 must be positive";
  if (!(c.I0 > 0) || !(c.wavelength > 0)) return "I0 and wavelength must be positive";
  if (!(c.kappa_esc > 0) || c.kappa_tnsa < 0 || c.sigma_dtheta < 0) return "bad reflux parameters";
  if (c.reflux_ke_frac < 0 || c.reflux_ke_frac >= 1) return "reflux_ke_frac must be in [0, 1)";
  if (!(c.brem_boost >= 1)) return "brem_boost must be >= 1";
  if (!(c.k_cut > 0) || !(c.table_emax > c.k_cut)) return "need 0 < k_cut < table_emax";
  if (c.table_shape != HYB_TABLE_CSBH && c.table_shape != HYB_TABLE_FLAT) return "unknown table shape";
  if (c.table_nT < 2 || c.table_nr < 2 || (double)c.table_nT * c.table_nr > 1e7) return "bad table size";
  if (!(c.e_min > c.k_cut)) return "e_min must exceed k_cut";
  if (c.tally_nE < 1 || c.tally_ntheta < 1 || !(c.tally_Ehi > c.tally_Elo) || !(c.tally_Elo > 0)) return "bad tally bins";
  if (c.series_len < 0) return "series_len must be >= 0";
  if (c.max_particles < 1 || c.max_particles > 2000000000LL) return "max_particles out of range";
  if ((c.physics & ~0x3FFu) != 0) return "unknown physics bits";
  if ((c.physics & HYB_PHYS_URBAN) && !(c.physics & HYB_PHYS_SCATTER))
    return "the Urban-type scatter replaces the Davies scatter: set HYB_PHYS_SCATTER too";
  if (c.physics & HYB_PHYS_DELTA) {
    if (!(c.physics & HYB_PHYS_ION)) return "delta rays need HYB_PHYS_ION";
    if (!(c.delta_cut > 0)) return "delta_cut must be positive";
  }
  if (c.eta_fixed < 0) return "eta_fixed must be >= 0";
  if (c.n_sub < 0 || c.n_sub > 1000) return "n_sub out of range";
  if (c.sort_every < 0) return "sort_every must be >= 0";
  if (c.n_extra < 0 || c.n_extra > 3) return "n_extra must be in [0, 3]";
  for (int k = 0; k < c.n_extra; ++k)
    if (!(c.extra_Z[k] >= 1) || !(c.extra_A[k] > 0) || !(c.extra_rho[k] > 0) || c.extra_I_ex[k] < 0)
      return "bad compound element";
  if (c.n_extra > 0 && (c.physics & HYB_PHYS_FSIGMA)) return "eq. F_sigma needs a single-element solid";
  for (int b : {c.bc_x, c.bc_y, c.bc_z})
    if (b != HYB_BC_REFLUX && b != HYB_BC_OPEN && b != HYB_BC_MIRROR && b != HYB_BC_PERIODIC)
      return "unknown boundary kind";
  if (c.bc_x == HYB_BC_PERIODIC) return "the x faces are the slab's: no periodic kind in x";
  if ((c.bc_y == HYB_BC_PERIODIC || c.bc_z == HYB_BC_PERIODIC) &&
      (c.physics & (HYB_PHYS_FIELDS | HYB_PHYS_EVOLVE_E | HYB_PHYS_EVOLVE_B)))
    return "periodic walls are for runs without field feedback";
  return "";
}

// The solid's elements: the first is (Z, A, rho, I_ex), then the extras.
struct Elem { double Z, A, rho, n, I; };
static std::vector<Elem> elements(const hyb_config& c) {
  std::vector<Elem> v;
  v.push_back(Elem{c.Z, c.A, c.rho, c.rho / (c.A * kAmu), c.I_ex > 0 ? c.I_ex : 11.0 * kE * c.Z});
  for (int k = 0; k < c.n_extra; ++k)
    v.push_back(Elem{c.extra_Z[k], c.extra_A[k], c.extra_rho[k], c.extra_rho[k] / (c.extra_A[k] * kAmu),
                     c.extra_I_ex[k] > 0 ? c.extra_I_ex[k] : 11.0 * kE * c.extra_Z[k]});
  return v;
}

// The compound of the heat update: one element is the plain solid; several
// are each taken as if they filled the cell at the total ion density.
static Mix make_mix(const hyb_config& c) {
  const std::vector<Elem> e = elements(c);
  Mix m{};
  m.n = (int)e.size();
  double n_t = 0.0, ne = 0.0;
  for (const Elem& x : e) { n_t += x.n; ne += x.Z * x.n; }
  m.ne = ne;
  for (int k = 0; k < m.n; ++k) {
    m.w[k] = e[k].Z * e[k].n / ne;
    m.x[k] = e[k].n / n_t;
    m.el[k] = m.n == 1 ? make_solid(e[k].Z, e[k].A, e[k].rho, e[k].n, c.lambda1, c.lambda2)
                       : make_solid(e[k].Z, e[k].A, n_t * e[k].A * kAmu, n_t, c.lambda1, c.lambda2);
  }
  return m;
}

static int n_sub_auto(const hyb_config& c) {
  const Mix mix = make_mix(c);
  double eta_max = 0.0;
  const double a = log10(c.T0), b = 9.0;
  for (int i = 0; i < 400; ++i) {
    const double T = i == 399 ? 1e9 : pow(10.0, a + i * (b - a) / 399.0);
    eta_max = fmax(eta_max, resistivity_mix(mix, T, T));
  }
  const double dt_max = 0.9 * kMu0 * c.dx * c.dx / (6.0 * eta_max);
  return std::max(1, (int)ceil(c.dt / dt_max));
}

static void set_units(RunDesc& h, double w_ref) {
  h.w_ref = w_ref;
  h.j_unit = kE * w_ref * kC / (h.dx * h.dx * h.dx) / kJScale;
  h.heat_unit = w_ref * kMec2 / kHeatScale;
  h.led_unit = w_ref * kMec2 / kLedScale;
  h.cnt_unit = w_ref / kLedScale;
}

static void fill_desc(hyb_run* r) {
  const hyb_config& c = r->cfg;
  RunDesc& h = r->h;
  h.nx = c.nx; h.ny = c.ny; h.nz = c.nz;
  h.ix_lo = (int)llround(c.x_lo / c.dx);
  h.ix_hi = (int)llround(c.x_hi / c.dx);
  h.precision = c.precision;
  h.physics = c.physics;
  h.seed = c.seed;
  h.nodes = (long long)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
  h.cells = (long long)c.nx * c.ny * c.nz;
  h.fd_sx = make_fastdiv((uint32_t)(c.nx + 1));
  h.fd_sy = make_fastdiv((uint32_t)(c.ny + 1));
  h.fd_w = make_fastdiv((uint32_t)(h.ix_hi - h.ix_lo));
  h.fd_ny = make_fastdiv((uint32_t)c.ny);
  h.capacity = c.max_particles;
  h.dx = c.dx; h.dt = c.dt;
  const double n_i = c.rho / (c.A * kAmu);
  const double I_ex = c.I_ex > 0 ? c.I_ex : 11.0 * kE * c.Z;
  const double a0 = 8.5e-6 * sqrt(c.I0 * c.wavelength * c.wavelength);
  const double cz = cz_of(c.Z);
  h.n_sub = c.n_sub > 0 ? c.n_sub : n_sub_auto(c);
  h.e_kick = -kE * c.dt / (2.0 * kMe * kC);
  h.b_rot = -kE * c.dt / (2.0 * kMe);
  h.cdt_dx = kC * c.dt / c.dx;
  const double e4 = kE * kE * kE * kE;
  // electron processes sum over the solid's elements: sums of Z n, Z^2 n and
  // n C_Z, and the logarithms averaged with the weights of their terms
  const std::vector<Elem> els = elements(c);
  double zn = 0.0, zn_lnI = 0.0, z2n = 0.0, z2n_lnD = 0.0, ncz = 0.0;
  for (const Elem& e : els) {
    zn += e.Z * e.n;
    zn_lnI += e.Z * e.n * log(e.I / kMec2);
    z2n += e.Z * e.Z * e.n;
    z2n_lnD += e.Z * e.Z * e.n * log(4.0 * kEps0 * kH * kC / (pow(e.Z, 1.0 / 3.0) * kE * kE));
    ncz += e.n * cz_of(e.Z);
  }
  const bool single = els.size() == 1;
  h.c_ion = (single ? c.Z * n_i : zn) * e4 * c.dt / (4.0 * kPi * kEps0 * kEps0 * kMe * kMe * kC * kC * kC);
  h.ln_iex = single ? log(I_ex / kMec2) : zn_lnI / zn;
  {  // delta rays: restricted loss prefactor (half of eq. stop_ion's), Moller depth
    const double re = kE * kE / (4.0 * kPi * kEps0 * kMec2);
    const double hwp = kHbar * sqrt((single ? c.Z * n_i : zn) * kE * kE / (kEps0 * kMe));
    const double I_eff = single ? I_ex : exp(h.ln_iex) * kMec2;
    h.d_cut = c.delta_cut / kMec2;
    h.c_rst = 0.5 * h.c_ion;
    h.d_lnI2 = 2.0 * h.ln_iex;
    h.d_dens0 = 2.0 * log(hwp / I_eff) - 1.0;
    h.d_u2min = exp(-h.d_dens0);
    h.k_mol = (single ? n_i * c.Z : zn) * 2.0 * kPi * re * re * kC * c.dt;
    h.spawn_cap = (c.physics & HYB_PHYS_DELTA) ? c.max_particles : 0;
  }
  h.k_brem = c.brem_boost * (single ? n_i * cz : ncz) * kC * c.dt;
  h.k_sub = (single ? n_i * cz : ncz) * kC * c.dt;
  h.inv_boost = 1.0 / c.brem_boost;
  h.c_dav = (single ? c.Z * c.Z * n_i : z2n) * e4 * c.dt / (2.0 * kPi * kEps0 * kEps0 * kMe * kMe * kC * kC * kC);
  h.l_dav = single ? 4.0 * kEps0 * kH * kC / (pow(c.Z, 1.0 / 3.0) * kE * kE) : exp(z2n_lnD / z2n);
  {  // Urban-type scatter: per element 2 pi Z (Z + 1) n r_e^2 c dt and Moliere's
     // screening A = 1.13 (alpha Z^1/3 / (2 0.88534 u))^2 (1 + 3.76 (alpha Z)^2 / (1.13 beta^2))
    const double re = kE * kE / (4.0 * kPi * kEps0 * kMec2);
    const double alpha = kE * kE / (4.0 * kPi * kEps0 * kHbar * kC);
    h.u_n = (int)els.size();
    for (int j = 0; j < h.u_n; ++j) {
      const double Z = els[j].Z;
      const double t = alpha * cbrt(Z) / (2.0 * 0.88534);
      h.u_k1[j] = 2.0 * kPi * Z * (Z + 1.0) * els[j].n * re * re * kC * c.dt;
      h.u_ca[j] = 1.13 * t * t;
      h.u_cb[j] = 3.76 * alpha * alpha * Z * Z / 1.13;
    }
  }
  h.eps_esc = c.kappa_esc * a0;
  h.du_tnsa = c.kappa_tnsa * a0;
  h.reflux_ke_mode = c.reflux_ke_frac > 0 ? 1 : 0;
  h.keep_frac = 1.0 - c.reflux_ke_frac;
  h.sigma_dth = c.sigma_dtheta;
  h.bc[0] = c.bc_x; h.bc[1] = c.bc_y; h.bc[2] = c.bc_z;
  h.e_min = c.e_min / kMec2;
  h.tab_nT = c.table_nT;
  h.tab_nr = c.table_nr;
  h.tab_kcut = c.k_cut / kMec2;
  h.tab_ln_kcut = log(c.k_cut / kMec2);
  h.tab_s_scale = (c.table_nT - 1) / log(c.table_emax / c.k_cut);
  h.nE = c.tally_nE;
  h.nth = c.tally_ntheta;
  h.series_len = c.series_len;
  h.ln_Elo = log(c.tally_Elo / kMec2);
  h.e_bin_scale = c.tally_nE / log(c.tally_Ehi / c.tally_Elo);
  h.Ethr = c.tally_Ethr / kMec2;
  h.solid = make_solid(c.Z, c.A, c.rho, n_i, c.lambda1, c.lambda2);
  h.mix = make_mix(c);
  h.eta_fixed = c.eta_fixed;
  h.sort_every = c.sort_every;
  h.ntx = (c.nx + kTile - 1) / kTile;
  h.nty = (c.ny + kTile - 1) / kTile;
  h.ntz = (c.nz + kTile - 1) / kTile;
  h.ntiles = h.ntx * h.nty * h.ntz;
  h.scan_nblk = (h.ntiles + kScanTile - 1) / kScanTile;
  h.fd_gx = make_fastdiv((uint32_t)(c.nx >> 2) + 1);
  h.fd_gy = make_fastdiv((uint32_t)(c.ny >> 2) + 1);
  h.fd_tx = make_fastdiv((uint32_t)h.ntx);
  h.fd_ty = make_fastdiv((uint32_t)h.nty);
  h.hist_stride = (long long)hist_stride(c);
  set_units(h, r->w_ref > 0 ? r->w_ref : 1.0);
  r->solid_cells = (int64_t)(h.ix_hi - h.ix_lo) * c.ny * c.nz;
}

static void point_desc(hyb_run* r) {
  char* b = (char*)r->base;
  const Layout& L = r->lay;
  RunDesc& h = r->h;
  for (int d = 0; d < 3; ++d) {
    h.E[d] = b + L.off_E[d];
    h.B[d] = b + L.off_B[d];
    h.J[d] = (long long*)(b + L.off_J[d]);
    h.Jacc[d] = (long long*)(b + L.off_Jacc[d]);
  }
  h.heat_acc = (long long*)(b + L.off_heat_acc);
  h.tstamp = (int*)(b + L.off_stamp);
  h.tdirty = (int*)(b + L.off_dirty);
  h.pj = b + L.off_pj;
  h.ph = (long long*)(b + L.off_ph);
  h.Te = (double*)(b + L.off_Te);
  h.Ti = (double*)(b + L.off_Ti);
  for (int k = 0; k < 2; ++k) h.eta[k] = (double*)(b + L.off_eta[k]);
  h.ion_heat = (long long*)(b + L.off_heat);
  h.fsig = b + L.off_fsig;
  for (int k = 0; k < 2; ++k) {
    PartPtrs& p = h.p[k];
    p.cell = (uint32_t*)(b + L.off_part[k][0]);
    p.ox = b + L.off_part[k][1]; p.oy = b + L.off_part[k][2]; p.oz = b + L.off_part[k][3];
    p.ux = b + L.off_part[k][4]; p.uy = b + L.off_part[k][5]; p.uz = b + L.off_part[k][6];
    p.wn = b + L.off_part[k][7]; p.tau = b + L.off_part[k][8];
    p.id = (uint32_t*)(b + L.off_part[k][9]);
    p.taud = b + L.off_part[k][10];
  }
  h.sp_cell = (uint32_t*)(b + L.off_sp_cell);
  h.sp_pid = (uint32_t*)(b + L.off_sp_pid);
  for (int f = 0; f < 7; ++f) h.sp_f[f] = b + L.off_sp_f[f];
  h.sp_cnt = (unsigned*)(b + L.off_sp_cnt);
  h.sp_start = (unsigned*)(b + L.off_sp_start);
  h.sp_blk = (unsigned*)(b + L.off_sp_blk);
  h.sp_grp = (unsigned*)(b + L.off_sp_grp);
  h.sp_gpid = (unsigned*)(b + L.off_sp_gpid);
  h.tab_X = b + L.off_tabX;
  h.tab_SIG = b + L.off_tabSIG;
  h.tab_SUB = b + L.off_tabSUB;
  h.acc_led = (long long*)(b + L.off_acc_led);
  h.acc_hist = (long long*)(b + L.off_acc_hist);
  h.events = (long long*)(b + L.off_events);
  h.tot_led = (double*)(b + L.off_tot_led);
  h.tot_led_c = (double*)(b + L.off_tot_led_c);
  h.tot_hist = (double*)(b + L.off_tot_hist);
  h.tot_hist_c = (double*)(b + L.off_tot_hist_c);
  h.series = (double*)(b + L.off_series);
  h.ctr = (Counters*)(b + L.off_ctr);
  h.src = (const SourceDesc*)(b + L.off_src);
  h.tile_cnt = (unsigned*)(b + L.off_tile_cnt);
  h.tile_start = (unsigned*)(b + L.off_tile_start);
  h.chunk_home = (int*)(b + L.off_chunk_home);
  h.chunk_base = (unsigned*)(b + L.off_chunk_base);
  h.far_off = (unsigned*)(b + L.off_far);
  h.scan_blk = (unsigned*)(b + L.off_scan_blk);
  h.red = (double*)(b + L.off_red);
}

static hyb_status upload_desc(hyb_run* r) {
  HIPCHK(r, hipMemcpyAsync(r->d_desc, &r->h, sizeof(RunDesc), hipMemcpyHostToDevice, r->stream));
  HIPCHK(r, hipStreamSynchronize(r->stream));
  return HYB_OK;
}

static void* dev_alloc(const hyb_device& d, size_t bytes) {
  if (d.alloc) return d.alloc(bytes, d.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

static void dev_free(const hyb_device& d, void* p) {
  if (!p) return;
  if (d.free) d.free(p, d.user);
  else (void)hipFree(p);
}

// Launch plans of a batch.  Particle plans get a multiple of 8 blocks per run
// so the XCD split inside the particle kernel stays aligned.
struct PlanSpec { std::vector<BlockMap> zero, inject, particle, gather, grid, cells, fin, adv, scan, scan1; };

static void add_run_plans(PlanSpec& ps, int run, const RunDesc& h) {
  auto add = [&](std::vector<BlockMap>& v, int nb) {
    for (int b = 0; b < nb; ++b) v.push_back(BlockMap{run, b, nb, 0});
  };
  const long long cap = h.capacity;
  add(ps.zero, clampi((h.ntiles + 1023) / 1024, 1, 1024));
  add(ps.inject, clampi((cap / 16 + 255) / 256, 1, 512));
  // the particle plan must start on a multiple of 8 blocks
  while (ps.particle.size() % 8) ps.particle.push_back(BlockMap{run, 0, 0, -1});
  int npb = clampi((cap + 255) / 256, 8, 4096);
  npb = (npb + 7) / 8 * 8;
  add(ps.particle, npb);
  add(ps.gather, clampi((long long)((h.ny >> 2) + 1) * ((h.nz >> 2) + 1) * gather_segments(h.nx), 1, 4096));
  add(ps.grid, clampi((h.nodes + 511) / 512, 1, 4096));
  const long long sc = (long long)(h.ix_hi - h.ix_lo) * h.ny * h.nz;
  add(ps.cells, clampi((sc + 255) / 256, 1, 4096));
  add(ps.fin, clampi((2LL * h.nE * h.nth + 4 + 255) / 256, 1, 256));
  add(ps.adv, 1);
  add(ps.scan, h.scan_nblk);
  add(ps.scan1, 1);
}

static hyb_status upload_plans(hyb_run* owner, hipStream_t s, const PlanSpec& ps, LaunchSet& L,
                               BlockMap** d_maps, size_t* maps_bytes, const hyb_device& dev) {
  std::vector<BlockMap> all;
  std::vector<std::pair<Plan*, const std::vector<BlockMap>*>> parts = {
      {&L.zero, &ps.zero}, {&L.inject, &ps.inject}, {&L.particle, &ps.particle}, {&L.gather, &ps.gather},
      {&L.grid, &ps.grid},
      {&L.cells, &ps.cells}, {&L.fin, &ps.fin}, {&L.adv, &ps.adv}, {&L.scan, &ps.scan},
      {&L.scan1, &ps.scan1}};
  std::vector<size_t> offs;
  for (auto& p : parts) {
    offs.push_back(all.size());
    all.insert(all.end(), p.second->begin(), p.second->end());
  }
  const size_t need = all.size() * sizeof(BlockMap);
  if (need > *maps_bytes) {
    if (*d_maps) dev_free(dev, *d_maps);
    *d_maps = (BlockMap*)dev_alloc(dev, need);
    if (!*d_maps) { *maps_bytes = 0; return fail(owner, HYB_ENOMEM, "block map allocation failed"); }
    *maps_bytes = need;
  }
  HIPCHK(owner, hipMemcpyAsync(*d_maps, all.data(), need, hipMemcpyHostToDevice, s));
  HIPCHK(owner, hipStreamSynchronize(s));
  for (size_t k = 0; k < parts.size(); ++k) {
    parts[k].first->map = *d_maps + offs[k];
    parts[k].first->nb = (int)parts[k].second->size();
  }
  return HYB_OK;
}

// Allocate and initialise a run's device state (no plans).
// eq. F_sigma of every cell from the temperatures on the device (1 outside
// the solid), in the run's precision.
static hipError_t refresh_fsig(hyb_run* r) {
  const hyb_config& c = r->cfg;
  const size_t cells = (size_t)r->h.cells;
  std::vector<double> Te(cells), Ti(cells), f(cells, 1.0);
  hipError_t e = hipMemcpy(Te.data(), r->h.Te, cells * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(Ti.data(), r->h.Ti, cells * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  for (int k = 0; k < c.nz; ++k)
    for (int j = 0; j < c.ny; ++j)
      for (int i = r->h.ix_lo; i < r->h.ix_hi; ++i) {
        const size_t q = i + (size_t)c.nx * (j + (size_t)c.ny * k);
        f[q] = f_sigma(r->h.solid, Ti[q], zstar(r->h.solid, Te[q]));
      }
  if (c.precision == HYB_FP64) return hipMemcpy(r->h.fsig, f.data(), cells * 8, hipMemcpyHostToDevice);
  std::vector<float> g(f.begin(), f.end());
  return hipMemcpy(r->h.fsig, g.data(), cells * 4, hipMemcpyHostToDevice);
}

static hyb_status create_run(const hyb_config* cfg, const hyb_device* dev, hyb_run** out) {
  if (!cfg || !dev || !out) return HYB_EINVAL;
  *out = nullptr;
  const std::string v = validate(*cfg);
  hyb_run* r = new hyb_run();
  r->cfg = *cfg;
  r->dev = *dev;
  r->stream = (hipStream_t)dev->stream;
  if (!v.empty()) {
    hyb_status st = fail(r, HYB_EINVAL, v);
    *out = r;
    return st;
  }
  hipError_t e = hipSetDevice(dev->device);
  if (e != hipSuccess) { *out = r; return fail(r, HYB_EDEVICE, hipGetErrorString(e)); }
  r->lay = make_layout(*cfg);
  r->bytes = r->lay.total;
  r->base = dev_alloc(r->dev, r->bytes);
  if (!r->base) { *out = r; return fail(r, HYB_ENOMEM, "device allocation failed"); }
  fill_desc(r);
  point_desc(r);
  r->d_desc = (RunDesc*)((char*)r->base + r->lay.off_desc);
  // tables
  build_brem_table(cfg->k_cut, cfg->table_emax, cfg->table_nT, cfg->table_nr, cfg->table_shape, r->tabX,
                   r->tabSIG, r->tabSUB);
  const hyb_config& c = *cfg;
  const size_t ncells = (size_t)r->h.cells, nodes = (size_t)r->h.nodes;
  *out = r;
  // zero everything, then fill tables and the initial solid
  HIPCHK(r, hipMemsetAsync(r->base, 0, r->bytes, r->stream));
  std::vector<double> subm(r->tabSUB.size());
  for (size_t j = 0; j < subm.size(); ++j) subm[j] = r->tabSUB[j] / kMec2;
  auto put_typed = [&](void* dst, const std::vector<double>& v) -> hipError_t {
    if (c.precision == HYB_FP64) return hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    std::vector<float> f(v.begin(), v.end());
    return hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
  };
  HIPCHK(r, hipStreamSynchronize(r->stream));
  HIPCHK(r, put_typed((void*)r->h.tab_X, r->tabX));
  HIPCHK(r, put_typed((void*)r->h.tab_SIG, r->tabSIG));
  HIPCHK(r, put_typed((void*)r->h.tab_SUB, subm));
  {
    std::vector<double> T(ncells, c.T0), eta(ncells, 0.0);
    const double e0 = c.eta_fixed > 0 ? c.eta_fixed
                                      : resistivity_mix(r->h.mix, c.T0, c.T0);
    for (int k = 0; k < c.nz; ++k)
      for (int j = 0; j < c.ny; ++j)
        for (int i = r->h.ix_lo; i < r->h.ix_hi; ++i) eta[i + (size_t)c.nx * (j + (size_t)c.ny * k)] = e0;
    HIPCHK(r, hipMemcpy(r->h.Te, T.data(), ncells * 8, hipMemcpyHostToDevice));
    HIPCHK(r, hipMemcpy(r->h.Ti, T.data(), ncells * 8, hipMemcpyHostToDevice));
    for (int k = 0; k < 2; ++k) HIPCHK(r, hipMemcpy(r->h.eta[k], eta.data(), ncells * 8, hipMemcpyHostToDevice));
  }
  HIPCHK(r, refresh_fsig(r));
  (void)nodes;
  Counters ctr{};
  ctr.active = 1;
  HIPCHK(r, hipMemcpy(r->h.ctr, &ctr, sizeof(ctr), hipMemcpyHostToDevice));
  return HYB_OK;
}

static void destroy_run(hyb_run* r) {
  if (!r) return;
  (void)hipStreamSynchronize(r->stream);
  if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
  if (r->cap_stream) (void)hipStreamDestroy(r->cap_stream);
  for (hipStream_t q : {r->side, r->side2})
    if (q) { (void)hipStreamSynchronize(q); (void)hipStreamDestroy(q); }
  for (hipEvent_t v : {r->ev_fork, r->ev_join, r->ev_join2})
    if (v) (void)hipEventDestroy(v);
  for (auto& p : r->ev_pool) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  if (r->d_maps) dev_free(r->dev, r->d_maps);
  if (r->base) dev_free(r->dev, r->base);
  delete r;
}

// ---------------------------------------------------------------------------
// sources
// ---------------------------------------------------------------------------
static hyb_status add_source(hyb_run* r, const hyb_source* s) {
  const hyb_config& c = r->cfg;
  if (!s) return fail(r, HYB_EINVAL, "null source");
  if ((int)r->srcs.size() >= kMaxSources) return fail(r, HYB_EINVAL, "too many sources");
  if (s->n_macro < 1) return fail(r, HYB_EINVAL, "n_macro must be >= 1");
  if (!(s->t_end > s->t_start) || s->t_start < 0) return fail(r, HYB_EINVAL, "empty injection window");
  if (!(s->T_hot > 0) || !(s->r_fwhm > 0) || !(s->half_angle >= 0) || s->half_angle > kPi)
    return fail(r, HYB_EINVAL, "bad source parameters");
  const double Ly = c.ny * c.dx, Lz = c.nz * c.dx, rr = 0.5 * s->r_fwhm;
  if (s->y0 - rr < 0 || s->y0 + rr >= Ly || s->z0 - rr < 0 || s->z0 + rr >= Lz)
    return fail(r, HYB_EINVAL, "spot leaves the slab face");
  if (r->scheduled + s->n_macro > c.max_particles) return fail(r, HYB_ENOSPACE, "sources exceed max_particles");
  const long long s0 = (long long)floor(s->t_start / c.dt + 0.5);
  const long long ns = std::max(1LL, (long long)floor((s->t_end - s->t_start) / c.dt + 0.5));
  if (s0 < r->host_step) return fail(r, HYB_ESTATE, "source starts before the current step");
  double w = s->weight;
  if (!(w > 0)) {
    if (!(s->eta_l2e > 0)) return fail(r, HYB_EINVAL, "eta_l2e must be positive");
    const double f_mean = 1.0 / (2.0 * log(2.0));
    const double energy = c.I0 * f_mean * (kPi * s->r_fwhm * s->r_fwhm / 4.0) * (s->t_end - s->t_start) * s->eta_l2e;
    w = energy / ((double)s->n_macro * s->T_hot);
  }
  if (!r->w_locked && r->host_step == 0) {
    r->w_ref = std::max(r->w_ref, w);
  }
  const double wref = r->w_ref > 0 ? r->w_ref : w;
  // the accumulator units are per w_ref; FP32-mixed runs round each current
  // contribution to a 32-bit integer before the sums, which bounds w / w_ref at 2
  const double wmax = c.precision == HYB_FP64 ? 64.0 : 2.0;
  if (w / wref > wmax) return fail(r, HYB_EINVAL, "source weight too large for the accumulator scale");
  SourceDesc d{};
  d.s0 = s0;
  d.ns = ns;
  d.base = s->n_macro / ns;
  d.rem = s->n_macro % ns;
  d.id0 = r->next_id;
  d.y0 = s->y0 / c.dx;
  d.z0 = s->z0 / c.dx;
  d.sig2 = (s->r_fwhm * s->r_fwhm / (8.0 * log(2.0))) / (c.dx * c.dx);
  d.t_hot = s->T_hot / kMec2;
  d.one_minus_cos = 1.0 - cos(s->half_angle);
  d.wn = w;   // absolute here; divided by w_ref when uploaded
  r->srcs.push_back(d);
  r->next_id += s->n_macro;
  r->scheduled += s->n_macro;
  return HYB_OK;
}

static hyb_status add_envelope(hyb_run* r, const hyb_envelope* e) {
  const hyb_config& c = r->cfg;
  if (!e) return fail(r, HYB_EINVAL, "null envelope");
  if ((int)r->srcs.size() >= kMaxSources) return fail(r, HYB_EINVAL, "too many sources");
  if (e->per_cell < 1 || !(e->t_fwhm > 0) || !(e->r_fwhm > 0) || !(e->g_min > 0) || e->g_min > 1 ||
      !(e->f_min > 0) || e->f_min > 1 || !(e->max_half_angle > 0) || e->max_half_angle > kPi ||
      !(e->eta_l2e > 0) || !(e->t_peak >= 0))
    return fail(r, HYB_EINVAL, "bad envelope parameters");
  // injecting face cells, k-major: f at the cell centre >= f_min
  std::vector<int> cells;
  for (int k = 0; k < c.nz; ++k)
    for (int j = 0; j < c.ny; ++j) {
      const double rr = hypot((j + 0.5) * c.dx - e->y0, (k + 0.5) * c.dx - e->z0);
      const double q = 2.0 * rr / e->r_fwhm;
      if (exp2(-q * q) >= e->f_min) cells.push_back(j | (k << 16));
    }
  if (cells.empty()) return fail(r, HYB_EINVAL, "no face cell reaches f_min");
  // injecting steps: g at the step's middle >= g_min (a contiguous run)
  auto g_of = [&](long long n) {
    const double q = 2.0 * ((n + 0.5) * c.dt - e->t_peak) / e->t_fwhm;
    return exp2(-q * q);
  };
  const double half = 0.5 * e->t_fwhm * sqrt(log2(1.0 / e->g_min));
  long long n = std::max(0LL, (long long)floor((e->t_peak - half) / c.dt) - 2);
  const long long n_end = (long long)floor((e->t_peak + half) / c.dt) + 3;
  while (n <= n_end && g_of(n) < e->g_min) ++n;
  const long long s0 = n;
  while (n <= n_end && g_of(n) >= e->g_min) ++n;
  const long long ns = n - s0;
  if (ns < 1) return fail(r, HYB_EINVAL, "no step reaches g_min");
  if (s0 < r->host_step) return fail(r, HYB_ESTATE, "source starts before the current step");
  const long long per_step = (long long)cells.size() * e->per_cell;
  if (r->scheduled + per_step * ns > c.max_particles)
    return fail(r, HYB_ENOSPACE, "sources exceed max_particles");
  // eq. N_cell where f = g = 1 (a cell-step of envelope fg carries sqrt(fg) times this)
  const double a0 = 8.5e-6 * sqrt(c.I0 * c.wavelength * c.wavelength);
  const double w = c.I0 * c.dx * c.dx * c.dt * e->eta_l2e / (a0 * kMec2 * e->per_cell);
  if (!r->w_locked && r->host_step == 0) r->w_ref = std::max(r->w_ref, w);
  const double wref = r->w_ref > 0 ? r->w_ref : w;
  const double wmax = c.precision == HYB_FP64 ? 64.0 : 2.0;
  if (w / wref > wmax) return fail(r, HYB_EINVAL, "source weight too large for the accumulator scale");
  int* dcells = (int*)((char*)r->base + r->lay.off_env) + r->srcs.size() * (size_t)c.ny * c.nz;
  HIPCHK(r, hipStreamSynchronize(r->stream));
  HIPCHK(r, hipMemcpy(dcells, cells.data(), cells.size() * 4, hipMemcpyHostToDevice));
  SourceDesc d{};
  d.kind = 1;
  d.s0 = s0;
  d.ns = ns;
  d.base = per_step;
  d.rem = 0;
  d.id0 = r->next_id;
  d.per_cell = e->per_cell;
  d.cells = dcells;
  d.y0 = e->y0 / c.dx;
  d.z0 = e->z0 / c.dx;
  d.rf = e->r_fwhm / c.dx;
  d.tp = e->t_peak / c.dt;
  d.tf = e->t_fwhm / c.dt;
  d.a0 = a0;
  d.cap = e->max_half_angle;
  d.wn = w;   // absolute here; divided by w_ref when uploaded
  r->srcs.push_back(d);
  r->next_id += per_step * ns;
  r->scheduled += per_step * ns;
  return HYB_OK;
}

static hyb_status add_beam(hyb_run* r, const hyb_beam* b) {
  const hyb_config& c = r->cfg;
  if (!b) return fail(r, HYB_EINVAL, "null beam");
  if ((int)r->srcs.size() >= kMaxSources) return fail(r, HYB_EINVAL, "too many sources");
  if (b->per_cell < 1 || !(b->energy > 0) || !(b->weight > 0) || !(b->t_start >= 0))
    return fail(r, HYB_EINVAL, "bad beam parameters");
  const long long s0 = (long long)floor(b->t_start / c.dt + 0.5);
  if (s0 < r->host_step) return fail(r, HYB_ESTATE, "source starts before the current step");
  const long long n = (long long)b->per_cell * c.ny * c.nz;
  if (r->scheduled + n > c.max_particles) return fail(r, HYB_ENOSPACE, "sources exceed max_particles");
  if (!r->w_locked && r->host_step == 0) r->w_ref = std::max(r->w_ref, b->weight);
  const double wref = r->w_ref > 0 ? r->w_ref : b->weight;
  const double wmax = c.precision == HYB_FP64 ? 64.0 : 2.0;
  if (b->weight / wref > wmax) return fail(r, HYB_EINVAL, "source weight too large for the accumulator scale");
  SourceDesc d{};
  d.kind = 2;
  d.s0 = s0;
  d.ns = 1;
  d.base = n;
  d.rem = 0;
  d.id0 = r->next_id;
  d.per_cell = b->per_cell;
  d.t_hot = b->energy / kMec2;
  d.wn = b->weight;   // absolute here; divided by w_ref when uploaded
  r->srcs.push_back(d);
  r->next_id += n;
  r->scheduled += n;
  return HYB_OK;
}

static hyb_status upload_sources(hyb_run* r) {
  if (r->w_ref <= 0) r->w_ref = 1.0;
  set_units(r->h, r->w_ref);
  std::vector<SourceDesc> v = r->srcs;
  for (auto& d : v) d.wn /= r->w_ref;
  r->h.nsrc = (int)v.size();
  HIPCHK(r, hipStreamSynchronize(r->stream));
  if (!v.empty())
    HIPCHK(r, hipMemcpy((void*)r->h.src, v.data(), v.size() * sizeof(SourceDesc), hipMemcpyHostToDevice));
  return upload_desc(r);
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------
static hyb_status ensure_single_plans(hyb_run* r) {
  if (r->L.particle.nb > 0) return HYB_OK;
  PlanSpec ps;
  add_run_plans(ps, 0, r->h);
  r->L.runs = r->d_desc;
  r->L.nruns = 1;
  r->L.sort = r->h.sort_every > 0;
  r->L.delta = (r->h.physics & PHYS_DELTA) != 0;
  r->L.urban = (r->h.physics & PHYS_URBAN) != 0;
  r->L.compound = r->h.mix.n > 1;
  if (!r->side) {
    HIPCHK(r, hipStreamCreateWithFlags(&r->side, hipStreamNonBlocking));
    HIPCHK(r, hipStreamCreateWithFlags(&r->side2, hipStreamNonBlocking));
    HIPCHK(r, hipEventCreateWithFlags(&r->ev_fork, hipEventDisableTiming));
    HIPCHK(r, hipEventCreateWithFlags(&r->ev_join, hipEventDisableTiming));
    HIPCHK(r, hipEventCreateWithFlags(&r->ev_join2, hipEventDisableTiming));
  }
  r->L.side = r->side;
  r->L.side2 = r->side2;
  r->L.ev_fork = r->ev_fork;
  r->L.ev_join = r->ev_join;
  r->L.ev_join2 = r->ev_join2;
  return upload_plans(r, r->stream, ps, r->L, &r->d_maps, &r->maps_bytes, r->dev);
}

static hyb_status step_direct(hyb_run* r, int32_t nsteps) {
  for (int32_t s = 0; s < nsteps; ++s) {
    LaunchSet L = r->L;
    if (r->timing) {
      if (r->ev_used >= r->ev_pool.size()) {
        hipEvent_t a, b;
        HIPCHK(r, hipEventCreate(&a));
        HIPCHK(r, hipEventCreate(&b));
        r->ev_pool.push_back({a, b});
      }
      L.ev_start = r->ev_pool[r->ev_used].first;
      L.ev_stop = r->ev_pool[r->ev_used].second;
      r->ev_used++;
    }
    launch_step(L, r->stream, r->cfg.precision, r->h.n_sub);
    HIPCHK(r, hipGetLastError());
  }
  return HYB_OK;
}

static hyb_status step_graph(hyb_run* r, int32_t nsteps) {
  if (!r->gexec) {
    if (!r->cap_stream) HIPCHK(r, hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    hipGraph_t g = nullptr;
    HIPCHK(r, hipStreamBeginCapture(r->cap_stream, hipStreamCaptureModeThreadLocal));
    LaunchSet L = r->L;
    launch_step(L, r->cap_stream, r->cfg.precision, r->h.n_sub);
    HIPCHK(r, hipStreamEndCapture(r->cap_stream, &g));
    HIPCHK(r, hipGraphInstantiate(&r->gexec, g, nullptr, nullptr, 0));
    HIPCHK(r, hipGraphDestroy(g));
  }
  for (int32_t s = 0; s < nsteps; ++s) HIPCHK(r, hipGraphLaunch(r->gexec, r->stream));
  return HYB_OK;
}

// ---------------------------------------------------------------------------
// the energy-partition model scan (Sec. III.B): input checks and the staged
// run shared by hyb_model_scan and its allocation-free variant
// ---------------------------------------------------------------------------
static const char* model_inputs_error(const hyb_model* m, const double* I0, const double* Z, int64_t n,
                                      const double* out) {
  if (!m) return "null model";
  if (n < 0 || n > (1LL << 28)) return "n out of range";
  if (n == 0) return nullptr;
  if (!I0 || !Z || !out) return "null array";
  if (!(m->wavelength > 0) || !(m->eta_l2e > 0) || !(m->r_fwhm > 0) || !(m->t_fwhm > 0) ||
      !(m->fg_mean > 0) || m->fg_mean > 1 || !(m->sqrt_fg_mean > 0) || m->sqrt_fg_mean > 1 ||
      !(m->kappa_esc > 0) || !(m->kappa_tnsa >= 0) || !(m->e_th > 0) || !(m->Lx > 0) || !(m->Ly > 0) ||
      !(m->Lz > 0) || !(m->theta_c >= 0) || !(m->theta_c < 0.5 * kPi) || !(m->eta_mean >= 0) ||
      !(m->n_i > 0) || m->nsteps < 1 || m->nsteps > 1000000)
    return "bad model inputs";
  for (int64_t i = 0; i < n; ++i)
    if (!(I0[i] > 0) || !std::isfinite(I0[i]) || !(Z[i] >= 1) || !(Z[i] < 200))
      return "scan point outside I0 > 0, 1 <= Z < 200";
  return nullptr;
}

// Inputs in, the model, outputs out, through the device staging buf (8 n
// doubles: I0, Z, then the 6 n results); waits for the stream.
static hipError_t model_scan_on(const hyb_model& m, const double* I0, const double* Z, int64_t n, double* out,
                                double* buf, hipStream_t s) {
  double* dI = buf;
  double* dZ = buf + n;
  double* dout = buf + 2 * n;
  hipError_t e = hipMemcpyAsync(dI, I0, n * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dZ, Z, n * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    launch_model(m, dI, dZ, n, dout, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 6 * n * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t w = hipStreamSynchronize(s);
  return e != hipSuccess ? e : w;
}

// Staging of hyb_model_scan_static: a file-scope device array, one copy per
// GPU for the life of the process (8 doubles per scan point, 4 MiB).  In
// host code the array's name is not a device address; the address of the
// current device's copy comes from hipGetSymbolAddress, looked up once per
// device and kept in scan_scratch_ptr.
constexpr int64_t kScanStaticMax = 1 << 16;
constexpr int kScanStaticDevices = 64;
static __device__ __align__(256) double scratch[8 * kScanStaticMax];
static double* scan_scratch_ptr[kScanStaticDevices];
static std::mutex scan_scratch_mu;

static hyb_status scan_scratch(int device, double** p) {
  std::lock_guard<std::mutex> lock(scan_scratch_mu);
  if (!scan_scratch_ptr[device]) {
    void* q = nullptr;
    HIPCHK(nullptr, hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
    scan_scratch_ptr[device] = (double*)q;
  }
  *p = scan_scratch_ptr[device];
  return HYB_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* hyb_status_string(hyb_status s) {
  switch (s) {
    case HYB_OK: return "ok";
    case HYB_EINVAL: return "invalid argument";
    case HYB_ENOMEM: return "out of memory";
    case HYB_ENOSPACE: return "particle capacity exceeded";
    case HYB_EDEVICE: return "device error";
    case HYB_ESTATE: return "invalid state";
    case HYB_ENUMERIC: return "non-finite value";
    case HYB_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* hyb_last_error(const hyb_run* run) { return run ? run->err.c_str() : g_err.c_str(); }

hyb_status hyb_model_scan(const hyb_model* m, const double* I0, const double* Z, int64_t n, double* out,
                          const hyb_device* dev) {
  if (const char* why = model_inputs_error(m, I0, Z, n, out)) return fail(nullptr, HYB_EINVAL, why);
  if (n == 0) return HYB_OK;
  hyb_device d{};
  if (dev) d = *dev;
  HIPCHK(nullptr, hipSetDevice(d.device));
  hipStream_t s = (hipStream_t)d.stream;
  const size_t bytes = (size_t)n * 8 * sizeof(double);
  double* buf = (double*)dev_alloc(d, bytes);
  if (!buf) return fail(nullptr, HYB_ENOMEM, "device allocation failed");
  const hipError_t e = model_scan_on(*m, I0, Z, n, out, buf, s);
  dev_free(d, buf);
  if (e != hipSuccess) return fail(nullptr, HYB_EDEVICE, std::string("hyb_model_scan: ") + hipGetErrorString(e));
  return HYB_OK;
}

hyb_status hyb_model_scan_static(const hyb_model* m, const double* I0, const double* Z, int64_t n,
                                 double* out, const hyb_device* dev) {
  if (const char* why = model_inputs_error(m, I0, Z, n, out)) return fail(nullptr, HYB_EINVAL, why);
  if (n > kScanStaticMax)
    return fail(nullptr, HYB_EINVAL, "n exceeds the static staging of hyb_model_scan_static (65536 points)");
  if (n == 0) return HYB_OK;
  hyb_device d{};
  if (dev) d = *dev;
  if (d.device < 0 || d.device >= kScanStaticDevices) return fail(nullptr, HYB_EINVAL, "device ordinal out of range");
  HIPCHK(nullptr, hipSetDevice(d.device));
  double* buf = nullptr;
  hyb_status st = scan_scratch(d.device, &buf);
  if (st != HYB_OK) return st;
  const hipError_t e = model_scan_on(*m, I0, Z, n, out, buf, (hipStream_t)d.stream);
  if (e != hipSuccess)
    return fail(nullptr, HYB_EDEVICE, std::string("hyb_model_scan_static: ") + hipGetErrorString(e));
  return HYB_OK;
}

void hyb_abi_sizes(int64_t sizes[9]) {
  sizes[0] = sizeof(hyb_config);
  sizes[1] = sizeof(hyb_source);
  sizes[2] = sizeof(hyb_device);
  sizes[3] = sizeof(hyb_tally_out);
  sizes[4] = sizeof(hyb_state);
  sizes[5] = sizeof(hyb_run_info);
  sizes[6] = sizeof(hyb_envelope);
  sizes[7] = sizeof(hyb_beam);
  sizes[8] = sizeof(hyb_model);
}

hyb_status hyb_footprint(const hyb_config* cfg, int64_t* bytes) {
  if (!cfg || !bytes) return HYB_EINVAL;
  if (!validate(*cfg).empty()) return HYB_EINVAL;
  *bytes = (int64_t)make_layout(*cfg).total;
  return HYB_OK;
}

hyb_status hyb_init(const hyb_config* cfg, const hyb_device* dev, hyb_run** out) {
  if (!out) return HYB_EINVAL;
  hyb_run* r = nullptr;
  hyb_status st = create_run(cfg, dev, &r);
  if (st != HYB_OK) {
    // the message stays reachable through hyb_last_error(NULL)
    destroy_run(r);
    *out = nullptr;
    return st;
  }
  st = upload_desc(r);
  if (st != HYB_OK) { destroy_run(r); *out = nullptr; return st; }
  *out = r;
  return HYB_OK;
}

hyb_status hyb_inject(hyb_run* r, const hyb_source* src) {
  if (!r) return HYB_EINVAL;
  if (r->eng) return fail(r, HYB_ESTATE, "engine runs take their sources at admission");
  hyb_status st = add_source(r, src);
  if (st != HYB_OK) return st;
  return upload_sources(r);
}

hyb_status hyb_inject_envelope(hyb_run* r, const hyb_envelope* env) {
  if (!r) return HYB_EINVAL;
  if (r->eng) return fail(r, HYB_ESTATE, "engine runs take their sources at admission");
  hyb_status st = add_envelope(r, env);
  if (st != HYB_OK) return st;
  return upload_sources(r);
}

hyb_status hyb_inject_beam(hyb_run* r, const hyb_beam* beam) {
  if (!r) return HYB_EINVAL;
  if (r->eng) return fail(r, HYB_ESTATE, "engine runs take their sources at admission");
  hyb_status st = add_beam(r, beam);
  if (st != HYB_OK) return st;
  return upload_sources(r);
}

hyb_status hyb_step(hyb_run* r, int32_t nsteps) {
  if (!r) return HYB_EINVAL;
  if (r->eng) return fail(r, HYB_ESTATE, "engine runs advance through hyb_engine_step");
  if (nsteps < 0) return fail(r, HYB_EINVAL, "nsteps < 0");
  if (nsteps == 0) return HYB_OK;
  if (!r->w_locked) {
    r->w_locked = true;
    if (r->w_ref <= 0) r->w_ref = 1.0;
    hyb_status st = upload_sources(r);
    if (st != HYB_OK) return st;
  }
  hyb_status st = ensure_single_plans(r);
  if (st != HYB_OK) return st;
  HIPCHK(r, hipSetDevice(r->dev.device));
  st = (r->use_graph && !r->timing) ? step_graph(r, nsteps) : step_direct(r, nsteps);
  if (st == HYB_OK) r->host_step += nsteps;
  return st;
}

hyb_status hyb_use_graph(hyb_run* r, int32_t on) {
  if (!r) return HYB_EINVAL;
  r->use_graph = on != 0;
  return HYB_OK;
}

hyb_status hyb_timing_enable(hyb_run* r, int32_t on) {
  if (!r) return HYB_EINVAL;
  r->timing = on != 0;
  return HYB_OK;
}

hyb_status hyb_timing_get(hyb_run* r, double* total_ms, int64_t* launches) {
  if (!r) return HYB_EINVAL;
  HIPCHK(r, hipStreamSynchronize(r->stream));
  for (size_t k = 0; k < r->ev_used; ++k) {
    float ms = 0.f;
    HIPCHK(r, hipEventElapsedTime(&ms, r->ev_pool[k].first, r->ev_pool[k].second));
    r->t_ms += ms;
    r->t_n += 1;
  }
  r->ev_used = 0;
  if (total_ms) *total_ms = r->t_ms;
  if (launches) *launches = r->t_n;
  r->t_ms = 0.0;
  r->t_n = 0;
  return HYB_OK;
}

hyb_status hyb_run_info_get(const hyb_run* r, hyb_run_info* info) {
  if (!r || !info) return HYB_EINVAL;
  const hyb_config& c = r->cfg;
  info->n_sub = r->h.n_sub;
  info->a0 = 8.5e-6 * sqrt(c.I0 * c.wavelength * c.wavelength);
  info->eps_esc = r->h.eps_esc * kMec2;
  info->n_i = r->h.solid.n_i;
  info->c_z = cz_of(c.Z);
  info->w_ref = r->h.w_ref;
  info->nodes = r->h.nodes;
  info->cells = r->h.cells;
  info->bytes = (int64_t)r->bytes;
  return HYB_OK;
}

hyb_status hyb_table_get(const hyb_run* r, double* X, double* SIG, double* SUB) {
  if (!r) return HYB_EINVAL;
  if (X) memcpy(X, r->tabX.data(), r->tabX.size() * 8);
  if (SIG) memcpy(SIG, r->tabSIG.data(), r->tabSIG.size() * 8);
  if (SUB) memcpy(SUB, r->tabSUB.data(), r->tabSUB.size() * 8);
  return HYB_OK;
}

hyb_status hyb_tally(hyb_run* r, hyb_tally_out* out) {
  if (!r || !out) return HYB_EINVAL;
  HIPCHK(r, hipSetDevice(r->dev.device));
  HIPCHK(r, hipStreamSynchronize(r->stream));
  const int nbin = r->cfg.tally_nE * r->cfg.tally_ntheta;
  std::vector<double> hist(2 * (size_t)nbin + 4);
  HIPCHK(r, hipMemcpy(hist.data(), r->h.tot_hist, hist.size() * 8, hipMemcpyDeviceToHost));
  if (out->hist_E) memcpy(out->hist_E, hist.data(), (size_t)nbin * 8);
  if (out->hist_N) memcpy(out->hist_N, hist.data() + nbin, (size_t)nbin * 8);
  for (int k = 0; k < 4; ++k) out->flow[k] = hist[2 * (size_t)nbin + k];
  double led[16];
  HIPCHK(r, hipMemcpy(led, r->h.tot_led, 16 * 8, hipMemcpyDeviceToHost));
  for (int k = 0; k < HYB_LEDGER_N; ++k) out->ledger[k] = led[k];
  long long ev[16];
  HIPCHK(r, hipMemcpy(ev, r->h.events, 16 * 8, hipMemcpyDeviceToHost));
  for (int k = 0; k < HYB_COUNTER_N; ++k) out->counters[k] = ev[k];
  if (out->series && r->cfg.series_len > 0)
    HIPCHK(r, hipMemcpy(out->series, r->h.series, (size_t)r->cfg.series_len * 8, hipMemcpyDeviceToHost));
  Counters ctr;
  HIPCHK(r, hipMemcpy(&ctr, r->h.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
  out->step = ctr.step;
  // kinetic energy and alive count of the resident particles
  int nb = clampi((ctr.n_total + 255) / 256, 1, kRedBlocks);
  const RunDesc* base = r->eng ? r->d_desc : r->d_desc;
  launch_kinetic(base, 0, nb, r->stream, r->cfg.precision);
  HIPCHK(r, hipGetLastError());
  HIPCHK(r, hipStreamSynchronize(r->stream));
  std::vector<double> red(2 * (size_t)nb);
  HIPCHK(r, hipMemcpy(red.data(), r->h.red, red.size() * 8, hipMemcpyDeviceToHost));
  double kin = 0.0, alive = 0.0;
  for (int b = 0; b < nb; ++b) { kin += red[2 * b]; alive += red[2 * b + 1]; }
  out->kinetic = kin * r->h.w_ref * kMec2;
  out->n_alive = (int64_t)llround(alive);
  out->conversion = led[HYB_L_INJECTED] > 0 ? led[HYB_L_PHOTON_THR] / led[HYB_L_INJECTED] : 0.0;
  if (out->counters[HYB_C_INJ_LOST] > 0) return fail(r, HYB_ENOSPACE, "scheduled electrons found no particle slot");
  return HYB_OK;
}

hyb_status hyb_get_state(hyb_run* r, hyb_state* st) {
  if (!r || !st) return HYB_EINVAL;
  HIPCHK(r, hipSetDevice(r->dev.device));
  HIPCHK(r, hipStreamSynchronize(r->stream));
  const hyb_config& c = r->cfg;
  Counters ctr;
  HIPCHK(r, hipMemcpy(&ctr, r->h.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
  const size_t n = (size_t)ctr.n_total;
  const size_t ts = c.precision == HYB_FP64 ? 8 : 4;
  const PartPtrs& P = r->h.p[ctr.cur];
  std::vector<uint32_t> cell(n), id(n);
  const size_t rec = 8 + 8 * ts;
  std::vector<char> recs, rawd;
  const int nf = (c.physics & HYB_PHYS_DELTA) ? 9 : 8;
  if (n) {
    recs.resize(n * rec);
    HIPCHK(r, hipMemcpy(recs.data(), P.cell, n * rec, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i) {
      memcpy(&cell[i], recs.data() + i * rec, 4);
      memcpy(&id[i], recs.data() + i * rec + 4, 4);
    }
    if (nf == 9) {
      rawd.resize(n * ts);
      HIPCHK(r, hipMemcpy(rawd.data(), P.taud, n * ts, hipMemcpyDeviceToHost));
    }
  }
  auto val = [&](int f, size_t i) -> double {
    const char* p = f == 8 ? rawd.data() + i * ts : recs.data() + i * rec + 8 + f * ts;
    if (ts == 8) { double v; memcpy(&v, p, 8); return v; }
    float v;
    memcpy(&v, p, 4);
    return (double)v;
  };
  size_t alive = 0;
  for (size_t i = 0; i < n; ++i) alive += cell[i] != kDead;
  st->step = ctr.step;
  st->next_id = r->next_id;
  st->delta_next = ctr.delta_next;
  if ((int64_t)alive > st->capacity) {
    st->n = (int64_t)alive;
    return fail(r, HYB_ENOSPACE, "state buffers too small");
  }
  size_t k = 0;
  const double mc = kMe * kC;
  for (size_t i = 0; i < n; ++i) {
    if (cell[i] == kDead) continue;
    const uint32_t cc = cell[i];
    if (st->pos) {
      st->pos[3 * k + 0] = (cell_i(cc) + val(0, i)) * c.dx;
      st->pos[3 * k + 1] = (cell_j(cc) + val(1, i)) * c.dx;
      st->pos[3 * k + 2] = (cell_k(cc) + val(2, i)) * c.dx;
    }
    if (st->mom) {
      st->mom[3 * k + 0] = val(3, i) * mc;
      st->mom[3 * k + 1] = val(4, i) * mc;
      st->mom[3 * k + 2] = val(5, i) * mc;
    }
    if (st->w) st->w[k] = val(6, i) * r->h.w_ref;
    if (st->tau) st->tau[k] = val(7, i);
    if (st->tau_d) st->tau_d[k] = nf == 9 ? val(8, i) : 0.0;
    if (st->id) st->id[k] = id[i];
    ++k;
  }
  st->n = (int64_t)k;
  const size_t nodes = (size_t)r->h.nodes, cells = (size_t)r->h.cells;
  auto get_typed = [&](double* dst, const void* srcp, size_t cnt) -> hipError_t {
    if (ts == 8) return hipMemcpy(dst, srcp, cnt * 8, hipMemcpyDeviceToHost);
    std::vector<float> f(cnt);
    hipError_t e = hipMemcpy(f.data(), srcp, cnt * 4, hipMemcpyDeviceToHost);
    for (size_t i = 0; i < cnt; ++i) dst[i] = f[i];
    return e;
  };
  for (int d = 0; d < 3; ++d) {
    if (st->E) HIPCHK(r, get_typed(st->E + d * nodes, r->h.E[d], nodes));
    if (st->B) HIPCHK(r, get_typed(st->B + d * nodes, r->h.B[d], nodes));
    if (st->J) {
      std::vector<long long> j(nodes);
      HIPCHK(r, hipMemcpy(j.data(), r->h.J[d], nodes * 8, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < nodes; ++i) st->J[d * nodes + i] = (double)j[i] * r->h.j_unit;
    }
  }
  if (st->Te) HIPCHK(r, hipMemcpy(st->Te, r->h.Te, cells * 8, hipMemcpyDeviceToHost));
  if (st->Ti) HIPCHK(r, hipMemcpy(st->Ti, r->h.Ti, cells * 8, hipMemcpyDeviceToHost));
  if (st->eta) HIPCHK(r, hipMemcpy(st->eta, r->h.eta[ctr.step & 1], cells * 8, hipMemcpyDeviceToHost));
  if (st->ion_heat) {
    std::vector<long long> q(cells);
    HIPCHK(r, hipMemcpy(q.data(), r->h.ion_heat, cells * 8, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < cells; ++i) st->ion_heat[i] = (double)q[i] * r->h.heat_unit;
  }
  return HYB_OK;
}

hyb_status hyb_set_state(hyb_run* r, const hyb_state* st) {
  if (!r || !st) return HYB_EINVAL;
  if (r->eng) return fail(r, HYB_ESTATE, "engine runs do not take a state");
  const hyb_config& c = r->cfg;
  if (st->n < 0 || st->n > c.max_particles) return fail(r, HYB_ENOSPACE, "too many particles for max_particles");
  const size_t n = (size_t)st->n;
  if (n && (!st->pos || !st->mom || !st->w || !st->tau || !st->id))
    return fail(r, HYB_EINVAL, "particle arrays missing");
  const bool delta = (c.physics & HYB_PHYS_DELTA) != 0;
  if (n && delta && !st->tau_d) return fail(r, HYB_EINVAL, "delta rays need tau_d");
  if (st->delta_next < 0 || st->delta_next >= (int64_t)kDeltaIdBit) return fail(r, HYB_EINVAL, "delta_next out of range");
  {
    // electrons the sources will still inject from st->step on must fit too
    int64_t later = 0;
    for (const SourceDesc& d : r->srcs)
      for (long long i = std::max(0LL, (long long)st->step - d.s0); i < d.ns; ++i)
        later += d.base + (i < d.rem ? 1 : 0);
    if ((int64_t)n + later > c.max_particles)
      return fail(r, HYB_ENOSPACE, "particles plus later injections exceed max_particles");
  }
  HIPCHK(r, hipSetDevice(r->dev.device));
  HIPCHK(r, hipStreamSynchronize(r->stream));
  // accumulator scale: the largest weight given, unless sources fixed it
  if (!r->w_locked) {
    double wm = 0.0;
    for (size_t i = 0; i < n; ++i) wm = std::max(wm, st->w[i]);
    if (r->srcs.empty() && wm > 0) r->w_ref = wm;
    else if (wm > 0) r->w_ref = std::max(r->w_ref, wm);
    if (r->w_ref <= 0) r->w_ref = 1.0;
    set_units(r->h, r->w_ref);
  }
  {
    const double wmax = (c.precision == HYB_FP64 ? 64.0 : 2.0) * r->w_ref;
    for (size_t i = 0; i < n; ++i)
      if (!(st->w[i] > 0) || st->w[i] > wmax) return fail(r, HYB_EINVAL, "particle weight outside (0, w_max]");
  }
  const size_t ts = c.precision == HYB_FP64 ? 8 : 4;
  std::vector<uint32_t> cell(n);
  const int nf = delta ? 9 : 8;
  std::vector<double> f[9];
  for (int k = 0; k < nf; ++k) f[k].resize(n);
  const int lo[3] = {r->h.ix_lo, 0, 0}, hi[3] = {r->h.ix_hi, c.ny, c.nz};
  for (size_t i = 0; i < n; ++i) {
    int ci[3];
    for (int d = 0; d < 3; ++d) {
      double X = st->pos[3 * i + d] / c.dx;
      const double Xr = nearbyint(X);
      if (fabs(X - Xr) < 1e-12 * fmax(1.0, fabs(X))) X = Xr;   // on a cell face: undo x/dx rounding
      double fl = floor(X);
      double o = X - fl;
      if (ts == 4 && (double)(float)o >= 1.0) { fl += 1.0; o = 0.0; }
      if (!(fl >= lo[d] && fl < hi[d])) return fail(r, HYB_EINVAL, "particle outside the slab box");
      ci[d] = (int)fl;
      f[d][i] = o;
    }
    cell[i] = pack_cell(ci[0], ci[1], ci[2]);
    for (int d = 0; d < 3; ++d) f[3 + d][i] = st->mom[3 * i + d] / (kMe * kC);
    f[6][i] = st->w[i] / r->w_ref;
    f[7][i] = st->tau[i];
    if (delta) f[8][i] = st->tau_d[i];
    for (int k = 3; k < nf; ++k)
      if (!std::isfinite(f[k][i])) return fail(r, HYB_ENUMERIC, "non-finite particle value");
  }
  const PartPtrs& P = r->h.p[0];
  auto put_typed = [&](void* d, const double* v, size_t cnt) -> hipError_t {
    if (ts == 8) return hipMemcpy(d, v, cnt * 8, hipMemcpyHostToDevice);
    std::vector<float> fl(v, v + cnt);
    return hipMemcpy(d, fl.data(), cnt * 4, hipMemcpyHostToDevice);
  };
  if (n) {
    const size_t rec = 8 + 8 * ts;
    std::vector<char> recs(n * rec);
    for (size_t i = 0; i < n; ++i) {
      char* q = recs.data() + i * rec;
      memcpy(q, &cell[i], 4);
      memcpy(q + 4, &st->id[i], 4);
      for (int k = 0; k < 8; ++k) {
        if (ts == 8) memcpy(q + 8 + 8 * k, &f[k][i], 8);
        else { const float v = (float)f[k][i]; memcpy(q + 8 + 4 * k, &v, 4); }
      }
    }
    HIPCHK(r, hipMemcpy(P.cell, recs.data(), n * rec, hipMemcpyHostToDevice));
    if (delta) HIPCHK(r, put_typed(P.taud, f[8].data(), n));
  }
  const size_t nodes = (size_t)r->h.nodes, cells = (size_t)r->h.cells;
  for (int d = 0; d < 3; ++d) {
    if (st->E) HIPCHK(r, put_typed(r->h.E[d], st->E + d * nodes, nodes));
    if (st->B) HIPCHK(r, put_typed(r->h.B[d], st->B + d * nodes, nodes));
    HIPCHK(r, hipMemset(r->h.J[d], 0, nodes * 8));
    HIPCHK(r, hipMemset(r->h.Jacc[d], 0, nodes * 8));
  }
  if (st->Te) HIPCHK(r, hipMemcpy(r->h.Te, st->Te, cells * 8, hipMemcpyHostToDevice));
  if (st->Ti) HIPCHK(r, hipMemcpy(r->h.Ti, st->Ti, cells * 8, hipMemcpyHostToDevice));
  if (st->eta)   // both buffers: the next step reads one, and a run without heating never writes the other
    for (int k = 0; k < 2; ++k) HIPCHK(r, hipMemcpy(r->h.eta[k], st->eta, cells * 8, hipMemcpyHostToDevice));
  if (st->Te || st->Ti) HIPCHK(r, refresh_fsig(r));
  HIPCHK(r, hipMemset(r->h.ion_heat, 0, cells * 8));
  HIPCHK(r, hipMemset(r->h.heat_acc, 0, cells * 8));
  // claims carry the step number, which a state may set back
  HIPCHK(r, hipMemset(r->h.tstamp, 0, (size_t)r->h.ntiles * 4));
  HIPCHK(r, hipMemset(r->h.tdirty, 0, (size_t)r->h.ntiles * 4));
  if (delta) HIPCHK(r, hipMemset(r->h.sp_cnt, 0, (size_t)r->h.ntiles * 4));
  HIPCHK(r, hipMemset(r->h.acc_led, 0, 16 * 8));
  HIPCHK(r, hipMemset(r->h.acc_hist, 0, hist_stride(c) * kHistCopies * 8));
  Counters ctr{};
  ctr.n_total = (long long)n;
  ctr.step = st->step;
  ctr.cur = 0;
  ctr.active = 1;
  ctr.delta_next = st->delta_next;
  HIPCHK(r, hipMemcpy(r->h.ctr, &ctr, sizeof(ctr), hipMemcpyHostToDevice));
  r->host_step = st->step;
  if (st->next_id > r->next_id) r->next_id = st->next_id;
  return upload_desc(r);
}

void hyb_free(hyb_run* r) {
  if (!r || r->eng) return;
  (void)hipSetDevice(r->dev.device);
  destroy_run(r);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving engine
// ---------------------------------------------------------------------------
struct hyb_engine {
  hyb_device dev{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  hipStream_t side = nullptr, side2 = nullptr;   // field sub-cycles, heating beside the sort
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  int64_t budget = 0, used = 0;
  int32_t max_runs = 0;
  RunDesc* d_descs[2] = {nullptr, nullptr};      // per precision: [max_runs]
  std::vector<hyb_run*> slots[2];                 // per precision
  LaunchSet L[2];
  BlockMap* d_maps[2] = {nullptr, nullptr};
  size_t maps_bytes[2] = {0, 0};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  bool dirty[2] = {true, true};
  int max_sub[2] = {1, 1};
  std::string err;
};

static hyb_status eng_fail(hyb_engine* e, hyb_status s, const std::string& m) {
  e->err = m;
  g_err = m;
  return s;
}

#define EHIPCHK(e, call)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return eng_fail((e), HYB_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

static hyb_status eng_rebuild(hyb_engine* e, int p) {
  PlanSpec ps;
  int maxsub = 1, nres = 0;
  for (int s = 0; s < e->max_runs; ++s) {
    hyb_run* r = e->slots[p][s];
    if (!r) continue;
    add_run_plans(ps, s, r->h);
    maxsub = std::max(maxsub, r->h.n_sub);
    ++nres;
  }
  if (e->gexec[p]) { (void)hipGraphExecDestroy(e->gexec[p]); e->gexec[p] = nullptr; }
  e->dirty[p] = false;
  e->max_sub[p] = maxsub;
  e->L[p] = LaunchSet{};
  if (nres == 0) return HYB_OK;
  e->L[p].side = e->side;
  e->L[p].side2 = e->side2;
  e->L[p].ev_fork = e->ev_fork;
  e->L[p].ev_join = e->ev_join;
  e->L[p].ev_join2 = e->ev_join2;
  e->L[p].runs = e->d_descs[p];
  e->L[p].nruns = e->max_runs;
  for (int s = 0; s < e->max_runs; ++s) {
    if (e->slots[p][s] && e->slots[p][s]->h.sort_every > 0) e->L[p].sort = true;
    if (e->slots[p][s] && (e->slots[p][s]->h.physics & PHYS_DELTA)) e->L[p].delta = true;
    if (e->slots[p][s] && (e->slots[p][s]->h.physics & PHYS_URBAN)) e->L[p].urban = true;
    if (e->slots[p][s] && e->slots[p][s]->h.mix.n > 1) e->L[p].compound = true;
  }
  hyb_run tmp;
  hyb_status st = upload_plans(&tmp, e->stream, ps, e->L[p], &e->d_maps[p], &e->maps_bytes[p], e->dev);
  if (st != HYB_OK) return eng_fail(e, st, tmp.err);
  // capture one tick of this precision group as a graph
  hipGraph_t g = nullptr;
  EHIPCHK(e, hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
  launch_step(e->L[p], e->cap_stream, p, maxsub);
  EHIPCHK(e, hipStreamEndCapture(e->cap_stream, &g));
  EHIPCHK(e, hipGraphInstantiate(&e->gexec[p], g, nullptr, nullptr, 0));
  EHIPCHK(e, hipGraphDestroy(g));
  return HYB_OK;
}

extern "C" {

hyb_status hyb_engine_create(const hyb_device* dev, int64_t hbm_budget, int32_t max_runs, hyb_engine** out) {
  if (!dev || !out || max_runs < 1 || max_runs > 4096 || hbm_budget < 0) return HYB_EINVAL;
  *out = nullptr;
  if (hipSetDevice(dev->device) != hipSuccess) return HYB_EDEVICE;
  hyb_engine* e = new hyb_engine();
  e->dev = *dev;
  e->stream = (hipStream_t)dev->stream;
  e->max_runs = max_runs;
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete e; return HYB_EDEVICE; }
    hbm_budget = (int64_t)(0.9 * (double)fr);
  }
  e->budget = hbm_budget;
  for (int p = 0; p < 2; ++p) {
    e->slots[p].assign(max_runs, nullptr);
    e->d_descs[p] = (RunDesc*)dev_alloc(e->dev, sizeof(RunDesc) * max_runs);
    if (!e->d_descs[p]) { hyb_engine_free(e); return HYB_ENOMEM; }
    if (hipMemset(e->d_descs[p], 0, sizeof(RunDesc) * max_runs) != hipSuccess) { hyb_engine_free(e); return HYB_EDEVICE; }
  }
  if (hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&e->side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&e->side2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_join2, hipEventDisableTiming) != hipSuccess) {
    hyb_engine_free(e);
    return HYB_EDEVICE;
  }
  *out = e;
  return HYB_OK;
}

hyb_status hyb_engine_admit(hyb_engine* e, const hyb_config* cfg, const hyb_source* srcs, int32_t nsrc,
                            int32_t nsteps, hyb_run** out) {
  if (!e || !cfg || !out || nsrc < 0 || nsrc > kMaxSources || (nsrc > 0 && !srcs) || nsteps < 1) return HYB_EINVAL;
  *out = nullptr;
  const std::string v = validate(*cfg);
  if (!v.empty()) return eng_fail(e, HYB_EINVAL, v);
  const int p = cfg->precision;
  int slot = -1;
  for (int s = 0; s < e->max_runs; ++s)
    if (!e->slots[0][s] && !e->slots[1][s]) { slot = s; break; }
  const int64_t need = (int64_t)make_layout(*cfg).total;
  if (slot < 0) return eng_fail(e, HYB_EBUSY, "no free slot");
  if (e->used + need > e->budget) return eng_fail(e, HYB_EBUSY, "footprint does not fit the budget now");
  hyb_device d = e->dev;
  d.stream = e->stream;
  hyb_run* r = nullptr;
  hyb_status st = create_run(cfg, &d, &r);
  if (st != HYB_OK) {
    e->err = r ? r->err : "create failed";
    destroy_run(r);
    return st;
  }
  for (int k = 0; k < nsrc; ++k) {
    st = add_source(r, &srcs[k]);
    if (st != HYB_OK) { e->err = r->err; destroy_run(r); return st; }
  }
  r->w_locked = true;
  if (r->w_ref <= 0) r->w_ref = 1.0;
  r->eng = e;
  r->slot = slot;
  r->nsteps_engine = nsteps;
  r->d_desc = e->d_descs[p] + slot;
  st = upload_sources(r);   // also writes the descriptor into the engine slot
  if (st != HYB_OK) { e->err = r->err; r->eng = nullptr; destroy_run(r); return st; }
  Counters ctr{};
  ctr.active = 1;
  ctr.steps_left = nsteps;
  if (hipMemcpy(r->h.ctr, &ctr, sizeof(ctr), hipMemcpyHostToDevice) != hipSuccess) {
    r->eng = nullptr; destroy_run(r); return eng_fail(e, HYB_EDEVICE, "counter upload failed");
  }
  e->slots[p][slot] = r;
  e->used += need;
  e->dirty[p] = true;
  *out = r;
  return HYB_OK;
}

hyb_status hyb_engine_step(hyb_engine* e, int32_t nticks) {
  if (!e || nticks < 0) return HYB_EINVAL;
  EHIPCHK(e, hipSetDevice(e->dev.device));
  for (int p = 0; p < 2; ++p)
    if (e->dirty[p]) {
      EHIPCHK(e, hipStreamSynchronize(e->stream));
      hyb_status st = eng_rebuild(e, p);
      if (st != HYB_OK) return st;
    }
  for (int32_t t = 0; t < nticks; ++t)
    for (int p = 0; p < 2; ++p)
      if (e->gexec[p]) EHIPCHK(e, hipGraphLaunch(e->gexec[p], e->stream));
  for (int p = 0; p < 2; ++p)
    for (hyb_run* r : e->slots[p])
      if (r) r->host_step += nticks;
  return HYB_OK;
}

hyb_status hyb_engine_poll(hyb_engine* e, hyb_run** done, int32_t cap, int32_t* ndone) {
  if (!e || !ndone || (cap > 0 && !done)) return HYB_EINVAL;
  EHIPCHK(e, hipStreamSynchronize(e->stream));
  int32_t k = 0;
  for (int p = 0; p < 2; ++p)
    for (hyb_run* r : e->slots[p]) {
      if (!r) continue;
      Counters ctr;
      EHIPCHK(e, hipMemcpy(&ctr, r->h.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
      if (!ctr.active) {
        if (k < cap) done[k] = r;
        ++k;
      }
    }
  *ndone = std::min(k, cap);
  return HYB_OK;
}

hyb_status hyb_engine_retire(hyb_engine* e, hyb_run* r) {
  if (!e || !r || r->eng != e) return HYB_EINVAL;
  EHIPCHK(e, hipStreamSynchronize(e->stream));
  const int p = r->cfg.precision;
  e->slots[p][r->slot] = nullptr;
  e->used -= (int64_t)r->bytes;
  e->dirty[p] = true;
  RunDesc zero{};
  EHIPCHK(e, hipMemcpy(e->d_descs[p] + r->slot, &zero, sizeof(RunDesc), hipMemcpyHostToDevice));
  r->eng = nullptr;
  r->stream = e->stream;
  destroy_run(r);
  return HYB_OK;
}

hyb_status hyb_engine_stats(const hyb_engine* e, int32_t* resident, int64_t* bytes_used, int64_t* budget) {
  if (!e) return HYB_EINVAL;
  int32_t n = 0;
  for (int p = 0; p < 2; ++p)
    for (hyb_run* r : e->slots[p]) n += r != nullptr;
  if (resident) *resident = n;
  if (bytes_used) *bytes_used = e->used;
  if (budget) *budget = e->budget;
  return HYB_OK;
}

void hyb_engine_free(hyb_engine* e) {
  if (!e) return;
  (void)hipSetDevice(e->dev.device);
  (void)hipStreamSynchronize(e->stream);
  for (int p = 0; p < 2; ++p) {
    for (hyb_run* r : e->slots[p])
      if (r) { r->eng = nullptr; destroy_run(r); }
    if (e->gexec[p]) (void)hipGraphExecDestroy(e->gexec[p]);
    if (e->d_maps[p]) dev_free(e->dev, e->d_maps[p]);
    if (e->d_descs[p]) dev_free(e->dev, e->d_descs[p]);
  }
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  for (hipStream_t q : {e->side, e->side2})
    if (q) { (void)hipStreamSynchronize(q); (void)hipStreamDestroy(q); }
  for (hipEvent_t v : {e->ev_fork, e->ev_join, e->ev_join2})
    if (v) (void)hipEventDestroy(v);
  delete e;
}

}  // extern "C"
