/*
 * hyb.h -- C ABI of the MI355X hybrid-PIC library.
 *
 * The library advances the hybrid particle-in-cell step of Morris, Robinson
 * and Ridgers, "Highly efficient conversion of laser energy to hard X-rays in
 * high intensity laser-solid simulations" (arXiv 2107.01723): hot
 * macro-electrons crossing a cold resistive solid (Sec. II, App. A, App. B).
 *
 * Conventions of every entry point:
 *  - Units are SI at the boundary (m, s, J, K, kg m^-3, W m^-2, T, V m^-1).
 *  - Nothing throws across the ABI; every call returns a hyb_status.  On an
 *    error the run keeps its previous state and hyb_last_error(run) holds a
 *    message.  Errors of work already enqueued on the device surface at the
 *    next synchronising call (hyb_tally, hyb_get_state) as HYB_EDEVICE.
 *  - The library owns all device memory of a run.  It allocates through the
 *    caller's allocator callback when one is given (hipMalloc otherwise) and
 *    frees it in hyb_free.  All host buffers belong to the caller.
 *  - Device work is enqueued on the caller's stream (hyb_device.stream, a
 *    hipStream_t; NULL = the default stream) and the call returns without
 *    waiting, except where a function says it synchronises.
 *  - A run is not thread-safe: calls on one run must be serialised.
 *
 * Grid layout used by hyb_state: nx*ny*nz cubic cells of side dx; nodes
 * (i, j, k), 0 <= i <= nx.  Every field component is an array of
 * (nx+1)*(ny+1)*(nz+1) doubles indexed i + (nx+1)*(j + (ny+1)*k), with the
 * Yee positions
 *   Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)     (j_h alike)
 *   Bx (i, j+1/2, k+1/2)   By (i+1/2, j, k+1/2)   Bz (i+1/2, j+1/2, k)
 * and entries past a staggered range are zero.  Cell arrays have nx*ny*nz
 * entries indexed i + nx*(j + ny*k).  The three components of E, B or j are
 * stored one after the other (component-major).
 */
#ifndef HYB_H
#define HYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HYB_OK = 0,
  HYB_EINVAL = 1,    /* an argument or configuration value is out of range */
  HYB_ENOMEM = 2,    /* device or host allocation failed */
  HYB_ENOSPACE = 3,  /* the particle capacity (max_particles) would be exceeded */
  HYB_EDEVICE = 4,   /* a HIP call failed */
  HYB_ESTATE = 5,    /* the call does not fit the run's current state */
  HYB_ENUMERIC = 6,  /* a non-finite value was found */
  HYB_EBUSY = 7      /* serving engine: no slot or not enough device memory now */
} hyb_status;

enum { HYB_FP64 = 0, HYB_FP32_MIXED = 1 };
enum { HYB_TABLE_CSBH = 0, HYB_TABLE_FLAT = 1 };

/* physics toggles (hyb_config.physics); HYB_PHYS_ALL is the method */
enum {
  HYB_PHYS_FIELDS = 1 << 0,    /* push in the gathered E and B */
  HYB_PHYS_ION = 1 << 1,       /* continuous ionisation loss, eq. (stop_ion) */
  HYB_PHYS_BREM = 1 << 2,      /* bremsstrahlung, optical-depth method (App. B) */
  HYB_PHYS_SCATTER = 1 << 3,   /* Davies elastic scatter (App. B) */
  HYB_PHYS_EVOLVE_E = 1 << 4,  /* E from eq. (Ampere_Maxwell) each sub-cycle */
  HYB_PHYS_EVOLVE_B = 1 << 5,  /* B from eq. (Faraday_Lens) */
  HYB_PHYS_HEAT = 1 << 6,      /* App. A heating, exchange and resistivity */
  HYB_PHYS_ALL = 0x7F,
  /* bremsstrahlung cross-sections enhanced by the background ionisation,
   * eq. (F_sigma), per cell from the start-of-step temperatures; not part
   * of HYB_PHYS_ALL */
  HYB_PHYS_FSIGMA = 1 << 7,
  /* delta rays (App. B): the ionisation loss splits at the energy
   * cfg.delta_cut given to a background electron; below it the restricted
   * continuous stopping power of App. B replaces eq. (stop_ion), above it
   * Moller scatter by the optical-depth method (a depth of its own per
   * electron, at most one delta ray per electron and step) adds the delta
   * ray as a new macro-electron at the parent's start-of-step position,
   * with the parent's weight, ids HYB_DELTA_ID_BIT + 0, 1, ... in the order
   * (4x4x4-cell tile of the birth cell, x fastest; parent id); a delta ray
   * below e_min stops at once (ledger term STOPPED, the cell's heat).  Only
   * with HYB_PHYS_ION; not part of HYB_PHYS_ALL. */
  HYB_PHYS_DELTA = 1 << 8,
  /* the paper's other elastic model (App. B, Urban's approach) in place of
   * the Davies scatter: the polar angle of a step is drawn from model
   * functions whose first two Legendre moments are those of Lewis theory,
   * exp(-v dt / lambda_1) and exp(-v dt / lambda_2), no displacement within
   * the step.  The transport mean free paths come from the screened
   * Rutherford cross-section (nucleus and atomic electrons, Z (Z + 1)) with
   * Moliere's screening angle, summed over the solid's elements; the model
   * function is a core a exp(-a (1 - cos theta)) plus an isotropic part of
   * weight w_i, (a, w_i) fixed by the two moments (w_i = 0 and the first
   * moment alone where the pair needs w_i < 0).  Same draws as the Davies
   * scatter (part, polar angle, azimuth).  Only with HYB_PHYS_SCATTER; not
   * part of HYB_PHYS_ALL. */
  HYB_PHYS_URBAN = 1 << 9
};

/* Boundary kind of each axis (hyb_config.bc_x, bc_y, bc_z); the x faces are
 * the slab's, the y and z faces the domain walls. */
enum {
  HYB_BC_REFLUX = 0,   /* escape above kappa_esc a0 m c^2, else reflux (Sec. II.A) */
  HYB_BC_OPEN = 1,     /* every electron that leaves escapes (ledger term ESCAPED) */
  HYB_BC_MIRROR = 2,   /* specular reflection without loss or turn */
  HYB_BC_PERIODIC = 3  /* y and z only (App. C's depth-dose setup): an electron that
                          leaves through one wall re-enters through the opposite one,
                          momentum unchanged.  The field solve keeps its mirror ghosts
                          and the current is not folded across the seam, so this kind
                          is for runs without field feedback: rejected with
                          HYB_PHYS_FIELDS, HYB_PHYS_EVOLVE_E or HYB_PHYS_EVOLVE_B */
};

/* ids of delta rays have this bit set; injected electrons' ids stay below it */
#define HYB_DELTA_ID_BIT 0x80000000u

/* energy ledger terms (hyb_tally_out.ledger), J */
enum {
  HYB_L_INJECTED = 0,     /* kinetic energy of injected electrons */
  HYB_L_FIELD_LOSS = 1,   /* work done by E against electrons */
  HYB_L_FIELD_GAIN = 2,   /* work done by E on electrons */
  HYB_L_IONISATION = 3,   /* continuous ionisation loss */
  HYB_L_STOPPED = 4,      /* energy of electrons removed below e_min */
  HYB_L_RAD_DISCRETE = 5, /* energy of emitted macro-photons */
  HYB_L_RAD_SUBCUT = 6,   /* continuous radiation below k_cut */
  HYB_L_ESCAPED = 7,      /* energy of escaping electrons */
  HYB_L_REFLUX = 8,       /* energy lost in reflux events */
  HYB_L_PHOTON_THR = 9,   /* photon energy at or above tally_Ethr (part of term 5) */
  HYB_L_RESIDUAL = 10,    /* rounding residual: change of the stored kinetic energy
                             that no process explains (elastic rotations, sub-cut
                             loss below the precision of the particle state) */
  HYB_LEDGER_N = 11
};

/* event counters (hyb_tally_out.counters) */
enum {
  HYB_C_INJECTED = 0, HYB_C_EMITTED = 1, HYB_C_REFLUX = 2, HYB_C_ESCAPED = 3,
  HYB_C_STOPPED = 4,
  HYB_C_DELTA = 5,        /* delta rays emitted (those below e_min included) */
  HYB_C_DELTA_LOST = 6,   /* delta rays that found no free particle slot: their
                             energy is booked as STOPPED in the birth cell */
  HYB_C_ESTEPS = 7,       /* electron-steps: the electrons alive at the start of
                             each completed step (that step's injections
                             included), summed over the steps */
  HYB_C_INJ_LOST = 8,     /* scheduled electrons that found no particle slot
                             (never expected: delta rays leave the slots of
                             the injections still to come free; hyb_tally
                             reports HYB_ENOSPACE if it is not zero) */
  HYB_COUNTER_N = 9
};

/* Run configuration (copied by hyb_init).  The solid is one element filling
 * the slab x_lo <= x < x_hi over the whole y, z extent of the grid (App. A
 * "solid"); x_lo and x_hi must lie on cell faces.  The slab is also the
 * particle box: electrons leaving it escape or reflux (Sec. II.A). */
typedef struct hyb_config {
  int32_t nx, ny, nz;       /* cells; nx < 2048, ny < 1024, nz < 2048 */
  double dx;                /* cell side [m] */
  double dt;                /* time step [s] */
  int32_t precision;        /* HYB_FP64 or HYB_FP32_MIXED */
  double Z, A, rho;         /* atomic number, molar mass [g/mol], density [kg/m^3] */
  double I_ex;              /* mean excitation energy [J]; 0 -> 11 eV * Z (Sec. III.B) */
  double x_lo, x_hi;        /* slab x-extent [m] */
  double T0;                /* initial electron and ion temperature [K] */
  double lambda1, lambda2;  /* reduced Lee-More fit parameters (App. A: 7, 3.5) */
  double I0;                /* peak laser intensity [W/m^2] -> a0, eq. (a0) */
  double wavelength;        /* laser wavelength [m] */
  double kappa_esc;         /* escape above kappa_esc a0 m c^2 (Sec. II.A: 2) */
  double kappa_tnsa;        /* reflux |p| loss kappa_tnsa a0 m c (Sec. II.A: 2.7e-3) */
  double sigma_dtheta;      /* reflux scatter range [rad] (Sec. II.A: 23 deg) */
  double reflux_ke_frac;    /* > 0: lose this fraction of kinetic energy per reflux
                               instead of the momentum loss above */
  double brem_boost;        /* cross-section multiplier B >= 1 (Sec. II.B: 10) */
  double k_cut;             /* lowest emitted photon energy [J] */
  int32_t table_shape;      /* HYB_TABLE_CSBH or HYB_TABLE_FLAT spectral shape */
  int32_t table_nT, table_nr; /* rows (electron energy) and columns (variate) */
  double table_emax;        /* top table energy [J] */
  double e_min;             /* electrons below this kinetic energy are removed [J] */
  int32_t tally_nE, tally_ntheta; /* photon tally bins (energy x angle to +x) */
  double tally_Elo, tally_Ehi;    /* log-uniform energy bins [J] */
  double tally_Ethr;        /* threshold of the conversion efficiency [J] (1 MeV) */
  int32_t series_len;       /* steps recorded in the per-step emission series */
  uint32_t seed;            /* run seed of the counter-based random stream */
  int64_t max_particles;    /* particle capacity */
  uint32_t physics;         /* HYB_PHYS_* bits */
  double eta_fixed;         /* > 0: hold the solid's resistivity at this value */
  int32_t n_sub;            /* field sub-cycles per step; 0 = from the stability scan */
  int32_t sort_every;       /* cell-sort and compact particles every this many steps; 0 = never */
  double delta_cut;         /* delta-ray cut [J] (App. B: 1 keV), > 0 with HYB_PHYS_DELTA */
  int32_t bc_x, bc_y, bc_z; /* HYB_BC_* per axis (HYB_BC_REFLUX is the paper's) */
  /* compound solid (App. A: several single-element solids share the cells):
   * n_extra further elements mixed into the slab with (Z, A, rho, I_ex) above.
   * Electron processes sum over the elements; heating follows the paper's
   * compound rule (n_e summed, 1/C averaged with weights Z n); each element's
   * Z*, Coulomb logarithm and resistivity are taken as if it filled the cell
   * at the total ion density, the resistivity is sum(x Z* eta)/sum(x Z*)
   * over the ion shares x, and the electron-ion exchange rates add with the
   * shares.  Not with HYB_PHYS_FSIGMA. */
  int32_t n_extra;          /* 0..3 */
  double extra_Z[3];        /* atomic numbers */
  double extra_A[3];        /* molar masses [g/mol] */
  double extra_rho[3];      /* partial mass densities [kg/m^3] */
  double extra_I_ex[3];     /* mean excitation energies [J]; 0 -> 11 eV * Z */
} hyb_config;

/* An injection source (App. B, Sec. II.B): n_macro electrons spread evenly
 * over the steps of [t_start, t_end), placed on the slab's front face in a
 * Gaussian spot truncated at f >= 1/2, with exponential kinetic energies of
 * mean T_hot and directions uniform in a cone about +x. */
typedef struct hyb_source {
  int64_t n_macro;
  double t_start, t_end;    /* [s] */
  double y0, z0;            /* spot centre [m] */
  double r_fwhm;            /* spot full width at half maximum [m] */
  double T_hot;             /* mean kinetic energy [J] */
  double half_angle;        /* cone half-angle [rad] */
  double eta_l2e;           /* laser-to-electron efficiency (weight rule) */
  double weight;            /* real electrons per macro-electron; 0 -> from I0 */
} hyb_source;

/* The paper's own injection (Sec. II.B, eq. N_cell, App. B): in every step
 * whose middle time t has g(t) = 2^-(2(t - t_peak)/t_fwhm)^2 >= g_min, each
 * face cell (transverse cell of the slab's front face) whose centre has
 * f = 2^-(2r/r_fwhm)^2 >= f_min (r from (y0, z0)) injects per_cell
 * macro-electrons, uniform over the cell's face, with exponential kinetic
 * energies of mean a m c^2, a = a0 sqrt(f g) (eq. a0 from cfg.I0 and
 * cfg.wavelength), directions uniform in a cone about +x of half-angle
 * min(max_half_angle, atan(sqrt(2/(gamma - 1)))) (Moore scaling), and the
 * weight of eq. N_cell: I0 f g dx^2 dt eta_l2e / (a m c^2 per_cell). */
typedef struct hyb_envelope {
  int32_t per_cell;         /* macro-electrons per face cell per step */
  double t_peak, t_fwhm;    /* temporal envelope [s] */
  double y0, z0, r_fwhm;    /* spatial envelope [m] */
  double g_min, f_min;      /* cut-offs (the paper: 0.1 and 0.5) */
  double max_half_angle;    /* cone cap [rad] (the paper: 20 deg) */
  double eta_l2e;           /* laser-to-electron efficiency */
} hyb_envelope;

/* A mono-energetic beam at normal incidence (the depth-dose benchmark of
 * App. C): at the step of t_start, per_cell macro-electrons in every face
 * cell of the slab's front (all ny x nz cells), uniform over the cell's face,
 * with kinetic energy `energy` along +x and `weight` real electrons each. */
typedef struct hyb_beam {
  int32_t per_cell;
  double t_start;           /* [s] */
  double energy;            /* [J] */
  double weight;            /* real electrons per macro-electron, > 0 */
} hyb_beam;

/* Inputs of the paper's energy-partition model (Sec. III.B): the injection
 * condensed into three macro-electrons (kinetic energy below e_th, from
 * e_th to the escape energy kappa_esc a0 m c^2, above it) integrated
 * through the continuous stopping powers of bremsstrahlung (eq. stop_brem),
 * ionisation (eq. stop_ion, I = 11 eV Z), reflux (eq. stop_tnsa) and the
 * resistive field (eq. stop_field). */
typedef struct hyb_model {
  double wavelength;        /* laser wavelength [m] (eq. a0) */
  double eta_l2e;           /* laser-to-electron efficiency */
  double r_fwhm, t_fwhm;    /* injection envelope [m], [s] */
  double fg_mean;           /* <fg> over the injecting cells and steps (0.41) */
  double sqrt_fg_mean;      /* <sqrt fg> (0.61): <eps_k> = a0 m c^2 <sqrt fg> */
  double kappa_esc, kappa_tnsa;
  double e_th;              /* X-ray threshold [J] (1 MeV) */
  double Lx, Ly, Lz;        /* target size [m]; the escaping electron runs to Lx */
  double theta_c;           /* half-angle of the current cone in eq. stop_field [rad] */
  double eta_mean;          /* typical resistivity <eta> [Ohm m] */
  double n_i;               /* ion density [m^-3] (the paper: 6e28) */
  int32_t nsteps;           /* fourth-order Runge-Kutta steps per macro-electron */
} hyb_model;

typedef void* (*hyb_alloc_fn)(size_t bytes, void* user);
typedef void (*hyb_free_fn)(void* ptr, void* user);

typedef struct hyb_device {
  int32_t device;           /* HIP device ordinal */
  void* stream;             /* hipStream_t for all enqueued work; NULL = default */
  hyb_alloc_fn alloc;       /* optional device allocator (NULL -> hipMalloc) */
  hyb_free_fn free;         /* its matching free */
  void* user;               /* passed to alloc/free */
} hyb_device;

/* Results copied out by hyb_tally.  Pointer members are caller-owned
 * buffers (NULL skips them); scalar members are filled in. */
typedef struct hyb_tally_out {
  double* hist_E;           /* [tally_nE*tally_ntheta] photon energy per bin [J],
                               energy index major */
  double* hist_N;           /* same bins, real photon number */
  double* series;           /* [series_len] photon energy >= tally_Ethr per step [J] */
  double flow[4];           /* under-range energy, number; over-range energy, number */
  double ledger[HYB_LEDGER_N];
  double kinetic;           /* kinetic energy of the electrons still alive [J] */
  double conversion;        /* ledger[PHOTON_THR] / ledger[INJECTED] (eta_e->gamma) */
  int64_t counters[HYB_COUNTER_N];
  int64_t n_alive;          /* electrons alive */
  int64_t step;             /* steps completed */
} hyb_tally_out;

/* Full state for checkpoint/restore and tests (host memory, SI). */
typedef struct hyb_state {
  int64_t n;                /* particles: set_state reads n; get_state writes n */
  int64_t capacity;         /* get_state: length of the particle buffers */
  double* pos;              /* [n*3] x, y, z per particle [m] */
  double* mom;              /* [n*3] momentum [kg m/s] */
  double* w;                /* [n] real electrons per macro-electron */
  double* tau;              /* [n] remaining optical depth to the next emission */
  uint32_t* id;             /* [n] particle ids (random-stream keys) */
  double* E;                /* [3*nodes] V/m */
  double* B;                /* [3*nodes] T */
  double* J;                /* [3*nodes] A/m^2, get only: the last step's hot current */
  double* Te;               /* [cells] K */
  double* Ti;               /* [cells] K */
  double* eta;              /* [cells] Ohm m */
  double* ion_heat;         /* [cells] J, get only: the last step's collisional deposit */
  int64_t step;             /* steps completed */
  int64_t next_id;          /* next particle id (set_state: ids of later sources) */
  double* tau_d;            /* [n] remaining optical depth to the next delta ray;
                               required by set_state with HYB_PHYS_DELTA, else may be NULL */
  int64_t delta_next;       /* delta rays numbered so far (next id HYB_DELTA_ID_BIT + this) */
} hyb_state;

/* Derived run quantities (for tests and reports). */
typedef struct hyb_run_info {
  int32_t n_sub;            /* field sub-cycles per step */
  double a0;                /* eq. (a0) */
  double eps_esc;           /* escape energy [J] */
  double n_i;               /* ion density [m^-3] */
  double c_z;               /* bremsstrahlung prefactor C_Z [m^2] */
  double w_ref;             /* weight of the fixed-point accumulator unit */
  int64_t nodes, cells;
  int64_t bytes;            /* device memory held by the run */
} hyb_run_info;

typedef struct hyb_run hyb_run;
typedef struct hyb_engine hyb_engine;

/* Validate cfg, build the bremsstrahlung tables, allocate the run on
 * dev->device and set the initial solid (T = T0, eta(T0), E = B = 0).
 * Synchronises the stream.  HYB_EINVAL for a bad configuration, HYB_ENOMEM
 * when the allocation fails. */
hyb_status hyb_init(const hyb_config* cfg, const hyb_device* dev, hyb_run** out);

/* Schedule an injection source; ids n..n+n_macro-1 go to its electrons in
 * step order.  No device work.  HYB_ENOSPACE when all sources together
 * exceed max_particles; HYB_EINVAL when the spot leaves the slab face, the
 * window is empty, or the macro-electron weight exceeds the accumulator
 * limit (the fixed-point unit w_ref is the largest weight scheduled before
 * the first step; later weights may reach 64 w_ref in FP64 and 2 w_ref in
 * FP32-mixed runs); HYB_ESTATE when the run already started past t_start. */
hyb_status hyb_inject(hyb_run* run, const hyb_source* src);

/* Schedule the envelope injection of hyb_envelope; it counts as a source
 * (at most 8 per run) and ids continue the run's counter in (step, cell,
 * electron) order.  No device work beyond uploading the cell list.
 * HYB_EINVAL for bad parameters or when no cell or step injects;
 * HYB_ENOSPACE when the schedule exceeds max_particles; HYB_ESTATE as for
 * hyb_inject. */
hyb_status hyb_inject_envelope(hyb_run* run, const hyb_envelope* env);

/* Schedule a hyb_beam; it counts as a source (at most 8 per run) and ids
 * continue the run's counter in (face cell k-major, electron) order.
 * HYB_EINVAL for bad parameters or a weight beyond the accumulator limit of
 * hyb_inject; HYB_ENOSPACE when the schedule exceeds max_particles;
 * HYB_ESTATE when the run already started past t_start. */
hyb_status hyb_inject_beam(hyb_run* run, const hyb_beam* beam);

/* Enqueue nsteps full hybrid-PIC steps (inject, push and collide, deposit,
 * Ohm + Faraday sub-cycles, heating, tallies; optional cell sort). */
hyb_status hyb_step(hyb_run* run, int32_t nsteps);

/* Copy out tallies, ledger, counters and the alive kinetic energy.
 * Synchronises the stream.  Returns HYB_ENOSPACE (with everything copied
 * out) if scheduled electrons found no particle slot (HYB_C_INJ_LOST). */
hyb_status hyb_tally(hyb_run* run, hyb_tally_out* out);

/* Copy the whole state to host buffers (particles in internal order).
 * HYB_ENOSPACE when st->capacity is too small (st->n holds the need).
 * Synchronises the stream. */
hyb_status hyb_get_state(hyb_run* run, hyb_state* st);

/* Replace particles, fields, temperatures, resistivity, step, next id and
 * delta-ray count (NULL field/cell pointers keep the current arrays).
 * Clears the step's current and heat buffers.  HYB_EINVAL when a weight is
 * not positive or exceeds the accumulator limit of hyb_inject, or when tau_d
 * is NULL with HYB_PHYS_DELTA.  Synchronises the stream. */
hyb_status hyb_set_state(hyb_run* run, const hyb_state* st);

hyb_status hyb_run_info_get(const hyb_run* run, hyb_run_info* info);

/* Copy the FP64 master bremsstrahlung table: X [nT*nr] (inverse CDF in
 * x = ln(k/k_cut)/ln(eps/k_cut)), SIG [nT] (sigma/C_Z), SUB [nT] (sub-cut
 * stopping / C_Z, J).  Any pointer may be NULL. */
hyb_status hyb_table_get(const hyb_run* run, double* X, double* SIG, double* SUB);

/* Kernel timing for roofline reports: when enabled, hyb_step records HIP
 * events around every launch of the particle kernel on the run's stream.
 * hyb_timing_get synchronises and returns the total milliseconds and count. */
hyb_status hyb_timing_enable(hyb_run* run, int32_t on);
hyb_status hyb_timing_get(hyb_run* run, double* total_ms, int64_t* launches);

/* Capture one step as a HIP graph and replay it in hyb_step (1) or launch
 * kernels directly (0, default). */
hyb_status hyb_use_graph(hyb_run* run, int32_t on);

/* Device bytes hyb_init would allocate for cfg. */
hyb_status hyb_footprint(const hyb_config* cfg, int64_t* bytes);

void hyb_free(hyb_run* run);

/* Message of the last failed call on this run; with run == NULL, of the last
 * failed call of this thread (e.g. hyb_init, which returns no handle). */
const char* hyb_last_error(const hyb_run* run);
const char* hyb_status_string(hyb_status s);

/* The energy-partition model of Sec. III.B at n scan points (host arrays
 * I0 [W/m^2] and Z, n each), one GPU thread per macro-electron.  out
 * (host, caller-owned, 6 n doubles, point-major) receives the fractions of
 * the injected hot-electron energy lost to: bremsstrahlung (all photons),
 * photons above e_th (eta_e->gamma, part of the first), ionisation,
 * reflux, the field, and escape.  Integration: for each macro-electron,
 * nsteps classical Runge-Kutta steps with u = ln(1 + eps / 1 keV) as the
 * independent variable from its energy down to zero, the state being the
 * path and the energy given to each mechanism; the escaping electron stops
 * where its path reaches Lx (state interpolated linearly between the two
 * steps around the crossing) and what it has not lost escapes.  dev may be
 * NULL (device 0, default stream).  Device buffers come from dev's
 * allocator (hipMalloc otherwise) and are freed before return.
 * Synchronous.  HYB_EINVAL for bad inputs (non-positive sizes or
 * intensities, Z < 1, nsteps outside [1, 1e6]); HYB_ENOMEM; HYB_EDEVICE. */
hyb_status hyb_model_scan(const hyb_model* m, const double* I0, const double* Z, int64_t n,
                          double* out, const hyb_device* dev);

/* hyb_model_scan for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and results, staged through a device array that the
 * library holds for the life of the process, one copy per GPU (4 MiB), so
 * no device allocation or free happens in the call.  Same arguments,
 * ownership and errors as hyb_model_scan, plus HYB_EINVAL when
 * n > 65536 points or dev->device is outside [0, 64).  The first call on a
 * device looks up that device's copy.  Calls that overlap on one GPU share
 * the array and race: serialise them.  Synchronous. */
hyb_status hyb_model_scan_static(const hyb_model* m, const double* I0, const double* Z, int64_t n,
                                 double* out, const hyb_device* dev);

/* sizeof of the ABI structs, for bindings to check their layouts:
 * config, source, device, tally_out, state, run_info, envelope, beam, model. */
void hyb_abi_sizes(int64_t sizes[9]);

/* ---------------- serving engine (continuous batching) -------------------
 * Independent runs share one device.  Each engine tick advances every
 * resident unfinished run by one step with batched kernels: one launch per
 * phase covers all resident runs, so runs admitted while others are running
 * overlap on the device.  Each tick is captured as a HIP graph and replayed
 * until the set of resident runs changes.  Results of a run are bitwise the
 * same alone and in any mix (integer accumulators, per-particle random
 * streams). */

/* hbm_budget: bytes the engine may hold for runs (0 = 90 % of free memory);
 * max_runs: resident run slots. */
hyb_status hyb_engine_create(const hyb_device* dev, int64_t hbm_budget, int32_t max_runs,
                             hyb_engine** out);

/* Admit a run with its sources and step count.  HYB_EBUSY when no slot is
 * free or its footprint does not fit the budget now; HYB_EINVAL for a bad
 * configuration.  The run handle serves hyb_tally / hyb_get_state /
 * hyb_run_info_get; it must not be passed to hyb_step or hyb_free. */
hyb_status hyb_engine_admit(hyb_engine* eng, const hyb_config* cfg, const hyb_source* srcs,
                            int32_t nsrc, int32_t nsteps, hyb_run** out);

/* Enqueue ticks; a run that has done its steps stops advancing. */
hyb_status hyb_engine_step(hyb_engine* eng, int32_t nticks);

/* Runs that have finished all their steps and are not yet retired
 * (synchronises the stream). */
hyb_status hyb_engine_poll(hyb_engine* eng, hyb_run** done, int32_t cap, int32_t* ndone);

/* Release a run's slot and memory; the handle becomes invalid. */
hyb_status hyb_engine_retire(hyb_engine* eng, hyb_run* run);

/* Resident runs and bytes in use. */
hyb_status hyb_engine_stats(const hyb_engine* eng, int32_t* resident, int64_t* bytes_used,
                            int64_t* budget);

void hyb_engine_free(hyb_engine* eng);

#ifdef __cplusplus
}
#endif
#endif /* HYB_H */
