// Internal definitions of the MI355X hybrid-PIC library: device-resident run
// descriptor, fixed-point accumulator scales, counter-based random numbers,
// table lookups and rotation helpers.  Shared by the kernels and the host
// runtime; never exposed through the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyb {

// ---- physical constants (CODATA 2018, SI) --------------------------------
constexpr double kC = 299792458.0;
constexpr double kE = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kHbar = 1.054571817e-34;
constexpr double kH = 6.62607015e-34;
constexpr double kKb = 1.380649e-23;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kPi = 3.14159265358979323846;
constexpr double kMec2 = kMe * kC * kC;

// ---- fixed-point accumulators --------------------------------------------
// Sums that many threads add into are 64-bit integers, so every sum is exact
// and independent of the order of the additions (runs are bitwise
// reproducible alone or batched, with any particle order).
//   ledger / tallies : 2^32 units per (w_ref m c^2) or per w_ref photons
//   hot current      : 2^40 units per (e w_ref c / dx^3)
//   collisional heat : 2^40 units per (w_ref m c^2)
constexpr double kLedScale = 4294967296.0;          // 2^32
constexpr double kJScale = 1099511627776.0;         // 2^40
constexpr double kHeatScale = 1099511627776.0;      // 2^40

enum { L_INJECTED = 0, L_FIELD_LOSS, L_FIELD_GAIN, L_ION, L_STOPPED, L_RAD_D, L_RAD_S,
       L_ESCAPED, L_REFLUX, L_PHOTON_THR, L_RESIDUAL, L_N };
enum { C_INJECTED = 0, C_EMITTED, C_REFLUX, C_ESCAPED, C_STOPPED, C_DELTA, C_DELTA_LOST, C_ESTEPS, C_INJ_LOST, C_N };

enum : uint32_t {
  PHYS_FIELDS = 1u << 0, PHYS_ION = 1u << 1, PHYS_BREM = 1u << 2, PHYS_SCATTER = 1u << 3,
  PHYS_EVOLVE_E = 1u << 4, PHYS_EVOLVE_B = 1u << 5, PHYS_HEAT = 1u << 6, PHYS_FSIGMA = 1u << 7,
  PHYS_DELTA = 1u << 8, PHYS_URBAN = 1u << 9
};

// delta rays: ids DELTA_ID_BIT + n; candidates of the energy sampler
constexpr uint32_t kDeltaIdBit = 0x80000000u;
constexpr int kDeltaTries = 32;

constexpr uint32_t kDead = 0xFFFFFFFFu;
constexpr int kMaxSources = 8;

// packed cell index: 11 bits x, 10 bits y, 11 bits z
__host__ __device__ __forceinline__ uint32_t pack_cell(int i, int j, int k) {
  return (uint32_t)i | ((uint32_t)j << 11) | ((uint32_t)k << 21);
}
__host__ __device__ __forceinline__ int cell_i(uint32_t c) { return (int)(c & 0x7FFu); }
__host__ __device__ __forceinline__ int cell_j(uint32_t c) { return (int)((c >> 11) & 0x3FFu); }
__host__ __device__ __forceinline__ int cell_k(uint32_t c) { return (int)(c >> 21); }

// Division of 32-bit unsigned values by a run constant d >= 1 through a
// multiply-high: q = (umulhi(t, m) + t) >> s with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1 (the round-up multiplier of Granlund and
// Montgomery), exact for every t < 2^32 with the sum taken in 64 bits.  The
// grid kernels turn flat node and cell indices into (i, j, k) with it
// instead of 64-bit divisions.
struct FastDiv {
  uint32_t m, s;
  __host__ __device__ __forceinline__ uint32_t div(uint32_t t) const;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t s = 0;
  while (((uint64_t)1 << s) < d) ++s;
  const uint64_t m = (((((uint64_t)1) << s) - d) << 32) / d + 1;
  return FastDiv{(uint32_t)m, s};
}

// Injection schedule and sampling parameters of one source (normalised units:
// lengths in cells, energies in m c^2).
struct SourceDesc {
  long long s0, ns, base, rem, id0;
  double y0, z0;          // spot centre [cells]
  double sig2;            // r_fwhm^2 / (8 ln 2) [cells^2]
  double t_hot;           // [m c^2]
  double one_minus_cos;   // 1 - cos(half angle); envelope: of the cap
  double wn;              // weight / w_ref; envelope: where f = g = 1
  // envelope injection (kind 1): per_cell electrons in each listed face cell;
  // beam (kind 2): per_cell electrons in every face cell, energy t_hot along +x
  int kind, per_cell;
  const int* cells;       // injecting face cells, j | k << 16, k-major
  double tp, tf;          // peak time and fwhm [steps]; step n is at n + 1/2
  double rf;              // spatial fwhm [cells]
  double a0;              // mean kinetic energy a0 sqrt(f g) [m c^2]
  double cap;             // cone half-angle cap [rad]
};

// Mutable per-run counters (device memory).
struct Counters {
  long long n_total;      // particle slots in use in the current buffer
  long long step;         // steps completed
  int cur;                // current particle buffer (0 or 1)
  int active;             // engine: 1 while the run still has steps to do
  long long steps_left;   // engine: steps still to do
  long long n_sorted;     // alive particles after the last compaction
  long long n_spawn;      // delta rays recorded this step (may exceed the record buffer)
  long long delta_next;   // delta rays numbered so far
};

// Structure-of-arrays particle storage: packed cell, offsets in the cell,
// momentum u = p / (m c), weight / w_ref, remaining optical depth, id.
struct PartPtrs {
  uint32_t* cell;
  void* ox; void* oy; void* oz;
  void* ux; void* uy; void* uz;
  void* wn; void* tau;
  uint32_t* id;
  void* taud;             // optical depth to the next delta ray (runs with delta rays)
};

// Material of the background solid (App. A), with the combinations of
// constants its per-cell formulas need, computed once per run.
struct Solid {
  double Z, A, rho, n_i, m_i, lambda1, lambda2;
  double z43;     // Z^(4/3)
  double lnR;     // ln(rho[g/cm^3] / (A Z)), More's reduced density
  double tf_c;    // Fermi temperature / n_e^(2/3): hbar^2 (3 pi^2)^(2/3) / (2 m_e k_B)
  double r0;      // ion-sphere radius (3 / (4 pi n_i))^(1/3)
  double th_c;    // tau_hot = th_c (k_B Te)^1.5 / (Z*^2 n_i lnL)
  double a_s;     // atomic screening length 1.4 a_B Z^(-1/3)
  double ln_as;   // ln(a_s m_e c / hbar), the complete-screening logarithm
  double tc_c;    // electron-ion exchange: 1 / tau = tc_c lnL / (Te m_i + Ti m_e)^1.5
  // products and quotients of constants the per-cell update multiplies by
  double t_ev;    // k_B / (e Z^(4/3)): Te [K] -> More's reduced temperature [eV]
  double ld_e;    // e^2 / (eps0 k_B): 1 / lambda_D^2 per n_e / T
  double ld_i;    // e^2 n_i / (eps0 k_B): the ions' share per Z*^2 / Ti
  double bc2;     // (e^2 / (12 pi eps0 k_B))^2: classical closest approach^2 * (T / Z*)^2
  double bq2;     // hbar^2 / (12 m_e k_B): de Broglie length^2 * T
  double r02;     // r0^2
  double inv_znk; // 1 / (Z n_i k_B)
  double tcold;   // lambda1 r0 sqrt(m_e / 3): tau_cold = tcold / sqrt(k_B Te)
  double eta_c;   // lambda2 m_e / (n_i e^2): eta = eta_c / (Z* tau)
};

// A compound solid (App. A): its elements, each as if it filled the cell at
// the total ion density n_t, with the weights of the heating rule and the
// ion shares.  One element: the plain solid.
constexpr int kMaxElems = 4;
struct Mix {
  int n;                    // elements
  double ne;                // sum of Z n over the elements (eq. Te_rise)
  double w[kMaxElems];      // Z n / ne: weights of 1 / C
  double x[kMaxElems];      // n / n_t: shares of the ion density
  Solid el[kMaxElems];
};

// Read-only description of one run (device memory; one per resident run).
struct RunDesc {
  int nx, ny, nz, ix_lo, ix_hi;
  FastDiv fd_sx, fd_sy;   // by nx + 1 and ny + 1 (node index -> i, j, k)
  FastDiv fd_w, fd_ny;    // by the slab width ix_hi - ix_lo and ny (solid cell index -> i, j, k)
  int n_sub, precision, nsrc;
  uint32_t physics, seed;
  long long nodes, cells, capacity;
  double dx, dt;
  // push and move
  double e_kick;      // du = e_kick * E  per half step  (q dt / (2 m c), q = -e)
  double b_rot;       // t  = b_rot * B / gamma          (q dt / (2 m))
  double cdt_dx;      // cells moved per unit beta
  // collisions (m c^2 units)
  double c_ion, ln_iex;
  double k_brem, k_sub, inv_boost;
  double c_dav, l_dav;
  // Urban-type scatter, per element: v dt / lambda_1 = sum k1 B1(A) / (u^2 beta),
  // A = ca (1 + cb / beta^2) / u^2 (Moliere), u = p / (m c)
  int u_n;
  double u_k1[kMaxElems], u_ca[kMaxElems], u_cb[kMaxElems];
  // boundaries
  double eps_esc, du_tnsa, keep_frac, sigma_dth, e_min;
  int reflux_ke_mode;
  int bc[3];          // boundary kind per axis: 0 reflux, 1 open, 2 mirror
  // tables (precision of the run)
  int tab_nT, tab_nr;
  double tab_ln_kcut, tab_s_scale, tab_kcut;
  const void* tab_X; const void* tab_SIG; const void* tab_SUB;
  // photon tally
  int nE, nth, series_len;
  double ln_Elo, e_bin_scale, Ethr;
  // fixed-point units
  double w_ref;
  double j_unit;      // A/m^2 per 2^-40 fixed unit of current
  double heat_unit;   // J per fixed unit of collisional heat
  double led_unit;    // J per fixed unit of the ledger
  double cnt_unit;    // photons per fixed unit of the number tally
  // solid (heat update, FP64): the first element, and the compound
  Solid solid;
  Mix mix;
  double eta_fixed;
  // delta rays (m c^2 units)
  double d_cut;       // cut
  double c_rst;       // restricted loss per step: c_rst * L / beta
  double d_lnI2;      // 2 ln(I / m c^2)
  double d_dens0;     // density effect: max(0, d_dens0 + ln (beta gamma)^2)
  double d_u2min;     // (beta gamma)^2 where the density effect starts: exp(-d_dens0)
  double k_mol;       // Moller depth per step: k_mol * J(x_c, gamma) / (beta (gamma - 1))
  // this step's delta rays, recorded by the particle kernel (record order is
  // the order of the atomics) and appended after the step's sort in the
  // order (tile of the birth cell, parent id)
  long long spawn_cap;
  uint32_t* sp_cell;        // [spawn_cap] packed birth cell
  uint32_t* sp_pid;         // [spawn_cap] parent id
  void* sp_f[7];            // [spawn_cap] ox oy oz ux uy uz wn (run precision)
  unsigned* sp_cnt;         // [ntiles] records per birth tile (cleared by the grouping)
  unsigned* sp_start;       // [ntiles] exclusive scan of sp_cnt
  unsigned* sp_blk;         // [scan_nblk] block sums of the scan
  unsigned* sp_grp;         // [spawn_cap] record index, grouped by tile
  unsigned* sp_gpid;        // [spawn_cap] parent id, grouped by tile
  // arrays
  void* E[3]; void* B[3];
  long long* J[3];
  double* Te; double* Ti;
  double* eta[2];           // resistivity: step n reads eta[n & 1], heating writes eta[(n + 1) & 1]
  void* fsig;               // [cells] eq. F_sigma of each cell (run precision), start of step
  long long* ion_heat;
  // The particle kernel's current and collisional heat: a workgroup that
  // first claims a tile in a step (tstamp[t] < step + 1, raised by its
  // atomicMax) stores that tile's LDS sums whole, as plain stores, in pj/ph;
  // every other contribution is added atomically into Jacc / heat_acc.  The
  // gather then sums, per node and cell, the accumulators and the partials
  // of the claimed tiles whose halos hold it into J / ion_heat, and clears
  // the accumulators it found non-zero.  Every atomic into them marks the
  // tile whose halo (or cell) it lands in, so that the gather reads the
  // accumulators of the nodes and cells of marked tiles only.
  long long* Jacc[3];
  long long* heat_acc;
  int* tstamp;              // [ntiles] step + 1 of the tile's last claim (0: never)
  int* tdirty;              // [ntiles] step + 1 of the last atomic into the tile's halo or cells
  void* pj;                 // [ntiles][3][kPjWords] current partials of the tiles (32-bit FP32, 64-bit FP64)
  long long* ph;            // [ntiles][64] heat partials of the tile's cells
  FastDiv fd_gx, fd_gy;     // by the gather's tile counts along x and y: (nx >> 2) + 1, (ny >> 2) + 1
  FastDiv fd_tx, fd_ty;     // by the tile counts ntx, nty
  PartPtrs p[2];
  Counters* ctr;
  const SourceDesc* src;
  long long* acc_led;       // [L_N] this step
  long long* acc_hist;      // [kHistCopies][hist_stride] this step: energy bins, number bins, flow
  long long hist_stride;    // >= 2*nE*nth + 4, in words
  long long* events;        // [C_N] whole run
  double* tot_led; double* tot_led_c;     // Kahan sum and compensation
  double* tot_hist; double* tot_hist_c;
  double* series;
  // counting sort of the particles by tile of 4x4x4 cells
  int sort_every;           // 0: never; S: after the particle kernel of every S-th step
  int ntx, nty, ntz, ntiles;
  int scan_nblk;            // scan blocks of kScanTile tiles
  unsigned* tile_cnt;       // [ntiles] electrons per destination tile
  unsigned* tile_start;     // [ntiles] exclusive scan of tile_cnt
  unsigned* scan_blk;       // [scan_nblk] block sums
  // Where the scatter puts each electron, fixed by the particle kernel's
  // counting: a chunk's electrons bound for tile t occupy
  // tile_start[t] + chunk_base[chunk][bin of t] + [0, count), and an electron
  // bound outside its chunk's neighbourhood sits at tile_start[t] + far_off[i].
  int* chunk_home;          // [chunks] first home tile of the chunk, the centre of its destination bins (none: kNoTile)
  unsigned* chunk_base;     // [chunks][kNbN]
  unsigned* far_off;        // [capacity]
  double* red;              // per-block partial sums for host-side reductions
};

constexpr int kTile = 4;           // tile edge in cells
// words per current component in a tile's partials: the nodes of its deposit
// halo (6^3) that the component reaches, staggered on one axis (6 x 5 x 5)
constexpr int kPjWords = (kTile + 2) * (kTile + 1) * (kTile + 1);
constexpr int kChunk = 256;        // electrons per chunk of the particle kernels (one workgroup)
constexpr int kNb = 5;             // destination tiles counted per chunk: home +-2 per axis
constexpr int kNbN = kNb * kNb * kNb;
constexpr int kNoTile = 0x7FFFFFFF;
// Photon tallies are accumulated in this many copies (workgroup b adds into
// copy b % kHistCopies), so that the memory-side atomics on the few hot bins
// of the spectrum do not all queue on one address; the step's finalisation
// sums the copies.
constexpr int kHistCopies = 32;
constexpr int kScanTile = 1024;    // tiles per scan block

// Segments of a row of tiles that the gather's workgroups take apart: rows
// of (nx >> 2) + 1 tiles in groups of 4, at most 8 groups per segment.
__host__ __device__ __forceinline__ uint32_t gather_segments(int nx) {
  const uint32_t ngr = ((uint32_t)(nx >> 2) + 1 + 3) / 4;
  return (ngr + 7) / 8;
}

// Does the step `step` end with a tile sort?
__host__ __device__ __forceinline__ bool sort_step(int sort_every, long long step) {
  return sort_every > 0 && (step + 1) % sort_every == 0;
}

// ---- Philox4x32-10 (Salmon et al., SC'11) ---------------------------------
struct U4 { uint32_t x, y, z, w; };

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(a, b);
#else
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
#endif
}

__host__ __device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = mulhi32(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = mulhi32(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__host__ __device__ __forceinline__ uint32_t FastDiv::div(uint32_t t) const {
  return (uint32_t)(((uint64_t)mulhi32(t, m) + t) >> s);
}

// 23-bit uniform strictly inside (0, 1), exact in FP32 and FP64
template <typename T>
__host__ __device__ __forceinline__ T uni(uint32_t x) {
  return ((T)(x >> 9) + (T)0.5) * (T)(1.0 / 8388608.0);
}

template <typename T> struct Uni4 { T a, b, c, d; };

template <typename T>
__host__ __device__ __forceinline__ Uni4<T> draws(uint32_t id, uint32_t seed, long long step, uint32_t slot) {
  U4 r = philox((uint32_t)step, slot, 0u, 0u, id, seed);
  return Uni4<T>{uni<T>(r.x), uni<T>(r.y), uni<T>(r.z), uni<T>(r.w)};
}

// Slots of the per-step draws: collisions; photon angles and new depth;
// reflux on x, y, z; injection; a delta ray's azimuth and new depth; the
// depths of a newborn delta ray (keyed by its own id); the sampler's
// candidates, two per slot from SLOT_DELTA_TRY on.
enum : uint32_t {
  SLOT_COLLIDE = 0, SLOT_PHOTON = 1, SLOT_REFLUX0 = 2, SLOT_INJ_A = 8, SLOT_INJ_B = 9,
  SLOT_DELTA_K = 12, SLOT_BIRTH = 13, SLOT_DELTA_TRY = 16
};

// ---- math in the run's precision ------------------------------------------
// Descriptor pointers are generic.  Kernels cast them to the global address
// space so that the compiler emits global rather than flat memory
// instructions: a flat access also counts against the LDS / scalar-load wait
// counter, so every wait for an LDS result would drain the HBM loads in
// flight as well.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> G(T* p) { return (gptr<T>)p; }

__device__ __forceinline__ void atomic_add_i64(long long* p, long long v) {
  __hip_atomic_fetch_add(G(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned atomic_add_u32(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(G(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bytes of one electron's record: cell and id (u32), then ox oy oz ux uy uz
// wn tau in the run's precision.  A record is contiguous, so the electrons
// that the sort moves to one tile reach HBM as whole lines.
template <typename T> constexpr long long kRec = 8 + 8 * (long long)sizeof(T);

// One field of the records: element i at the record base + i records + the
// field's offset.  Every field of a buffer shares the base, so the compiler
// sees one record's fields as neighbours and can merge their loads and stores.
template <typename T, typename U, int OFF>
struct RecField {
  gptr<char> b;
  __device__ __forceinline__ __attribute__((address_space(1))) U& operator[](long long i) const {
    return *(gptr<U>)(b + i * kRec<T> + OFF);
  }
};

// Particle arrays of one buffer, typed for the run's precision (the delta-ray
// depth is an array of its own).
template <typename T>
struct PartG {
  static constexpr int S = (int)sizeof(T);
  RecField<T, uint32_t, 0> cell;
  RecField<T, uint32_t, 4> id;
  RecField<T, T, 8> ox;
  RecField<T, T, 8 + S> oy;
  RecField<T, T, 8 + 2 * S> oz;
  RecField<T, T, 8 + 3 * S> ux;
  RecField<T, T, 8 + 4 * S> uy;
  RecField<T, T, 8 + 5 * S> uz;
  RecField<T, T, 8 + 6 * S> wn;
  RecField<T, T, 8 + 7 * S> tau;
  gptr<T> taud;
};
template <typename T>
__device__ __forceinline__ PartG<T> part_g(const PartPtrs& P) {
  const gptr<char> b = G((char*)P.cell);
  return PartG<T>{{b}, {b}, {b}, {b}, {b}, {b}, {b}, {b}, {b}, {b}, G((T*)P.taud)};
}

__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ float m_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double m_log1p(double x) { return log1p(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_cos(float x) { return cosf(x); }
__device__ __forceinline__ double m_cos(double x) { return cos(x); }
__device__ __forceinline__ float m_sin(float x) { return sinf(x); }
__device__ __forceinline__ double m_sin(double x) { return sin(x); }
// sine and cosine of x, and of 2 pi t (one argument reduction each)
__device__ __forceinline__ void m_sincos(float x, float& s, float& c) { sincosf(x, &s, &c); }
__device__ __forceinline__ void m_sincos(double x, double& s, double& c) { sincos(x, &s, &c); }
__device__ __forceinline__ void m_sincos2pi(float t, float& s, float& c) { sincospif(2.0f * t, &s, &c); }
__device__ __forceinline__ void m_sincos2pi(double t, double& s, double& c) { sincospi(2.0 * t, &s, &c); }
__device__ __forceinline__ float m_atan(float x) { return atanf(x); }
__device__ __forceinline__ double m_atan(double x) { return atan(x); }
__device__ __forceinline__ float m_acos(float x) { return acosf(x); }
__device__ __forceinline__ double m_acos(double x) { return acos(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ long long to_fixed(float x) { return __float2ll_rn(x); }
__device__ __forceinline__ long long to_fixed(double x) { return __double2ll_rn(x); }

// kinetic energy [m c^2] of u = p/(m c): u^2 / (1 + gamma), no cancellation
template <typename T>
__device__ __forceinline__ T kinetic(T u2, T g) { return u2 / ((T)1 + g); }

// |u| of kinetic energy e [m c^2]
template <typename T>
__device__ __forceinline__ T umag_of(T e) { return m_sqrt(e * (e + (T)2)); }

// Turn the unit direction (hx,hy,hz) by the polar angle of cosine c and sine
// s at azimuth phi = 2 pi t.  Basis: a = unit(h x e_m), e_m the axis of the
// smallest |h_i| (ties -> lowest index), b = h x a; d = c h + s (cos phi a +
// sin phi b).
template <typename T>
__device__ __forceinline__ void turn_unit(T hx, T hy, T hz, T c, T s, T t, T& dx, T& dy, T& dz) {
  const T ax_ = fabs(hx), ay_ = fabs(hy), az_ = fabs(hz);
  T ax, ay, az;
  if (ax_ <= ay_ && ax_ <= az_) { ax = (T)0; ay = hz; az = -hy; }        // h x x
  else if (ay_ <= az_)          { ax = -hz; ay = (T)0; az = hx; }        // h x y
  else                          { ax = hy; ay = -hx; az = (T)0; }        // h x z
  const T an = (T)1 / m_sqrt(ax * ax + ay * ay + az * az);
  ax *= an; ay *= an; az *= an;
  const T bx = hy * az - hz * ay, by = hz * ax - hx * az, bz = hx * ay - hy * ax;
  T cp, sp;
  m_sincos2pi(t, sp, cp);
  dx = c * hx + s * (cp * ax + sp * bx);
  dy = c * hy + s * (cp * ay + sp * by);
  dz = c * hz + s * (cp * az + sp * bz);
}

// Turn (ux,uy,uz) by the polar angle of cosine c and sine s at azimuth 2 pi t,
// keeping |u|.
template <typename T>
__device__ __forceinline__ void rotate_cs(T& ux, T& uy, T& uz, T c, T s, T t) {
  const T um = m_sqrt(ux * ux + uy * uy + uz * uz);
  const T inv = (T)1 / um;
  T dx, dy, dz;
  turn_unit(ux * inv, uy * inv, uz * inv, c, s, t, dx, dy, dz);
  const T dn = um / m_sqrt(dx * dx + dy * dy + dz * dz);
  ux = dx * dn; uy = dy * dn; uz = dz * dn;
}

// The same turn where |u| = um and 1/um = inv are known; the turned unit
// vector is used as computed (its length is 1 to rounding, which the ledger's
// rounding term books like any other).
template <typename T>
__device__ __forceinline__ void rotate_known(T& ux, T& uy, T& uz, T um, T inv, T c, T s, T t) {
  T dx, dy, dz;
  turn_unit(ux * inv, uy * inv, uz * inv, c, s, t, dx, dy, dz);
  ux = dx * um; uy = dy * um; uz = dz * um;
}

// The same turn by the polar angle dth.
template <typename T>
__device__ __forceinline__ void rotate(T& ux, T& uy, T& uz, T dth, T t) {
  T c, s;
  m_sincos(dth, s, c);
  rotate_cs(ux, uy, uz, c, s, t);
}

// ---- bremsstrahlung table lookups ------------------------------------------
template <typename T>
struct TableView {
  gptr<const T> X; gptr<const T> SIG; gptr<const T> SUB;
  int nT, nr;
  T ln_kcut, s_scale, kcut;
  __device__ __forceinline__ void row(T lneps, int& j, T& f) const {
    T s = s_scale * (lneps - ln_kcut);
    s = s > (T)0 ? s : (T)0;                    // also maps NaN to row 0
    s = s < (T)(nT - 1) ? s : (T)(nT - 1);
    int jj = (int)m_floor(s);
    jj = jj > nT - 2 ? nT - 2 : jj;
    j = jj; f = s - (T)jj;
  }
  // sigma / C_Z ; 0 at or below k_cut
  __device__ __forceinline__ T sigma(T eps, T lneps) const {
    if (!(eps > kcut)) return (T)0;
    int j; T f; row(lneps, j, f);
    return SIG[j] + f * (SIG[j + 1] - SIG[j]);
  }
  // sub-cut stopping / C_Z [m c^2]; eps itself at or below k_cut
  __device__ __forceinline__ T sub(T eps, T lneps) const {
    if (!(eps > kcut)) return eps;
    int j; T f; row(lneps, j, f);
    return SUB[j] + f * (SUB[j + 1] - SUB[j]);
  }
  // exponent of the inverse CDF at row j (fraction f) and variate r: the
  // photon energy is k_cut exp(x (ln eps - ln k_cut))
  __device__ __forceinline__ T x_at(int j, T f, T r) const {
    const T q = r * (T)(nr - 1);
    int i = (int)m_floor(q);
    i = i > nr - 2 ? nr - 2 : i;
    const T g = q - (T)i;
    const gptr<const T> r0 = X + (long long)j * nr;
    const gptr<const T> r1 = r0 + nr;
    const T x0 = r0[i] + g * (r0[i + 1] - r0[i]);
    const T x1 = r1[i] + g * (r1[i + 1] - r1[i]);
    return x0 + f * (x1 - x0);
  }
  // photon energy for an electron of kinetic energy eps > k_cut and variate r
  __device__ __forceinline__ T sample_k(T eps, T lneps, T r) const {
    int j; T f; row(lneps, j, f);
    return kcut * m_exp(x_at(j, f, r) * (lneps - ln_kcut));
  }
};

}  // namespace hyb
