"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module only *describes inputs*: grid sizes, materials, laser and
source parameters, seeds, and the random draws of the parameter scan.  It
holds none of the method's arithmetic (no physics, no tables, no RNG of the
method itself), so both the oracle and the product can import it without
sharing any computation.

All quantities are SI (m, s, J, K, kg m^-3, W m^-2) unless a key says
otherwise.  The workloads follow the paper's setup: hot electrons with an
exponential spectrum injected at the front face of a solid slab
(Sec. II.B and App. B), reflux boundaries (Sec. II.A), and laser intensities
of 1e20-1e22 W/cm^2.
"""
from __future__ import annotations

import copy
import math

import numpy as np

EV = 1.602176634e-19          # J per eV (exact, SI definition of e)
MEV = 1e6 * EV
KB = 1.380649e-23             # J/K (exact)

# Elements used by the paper's targets (Sec. III.A).  A in g/mol, rho in kg/m^3.
MATERIALS = {
    "Al": dict(Z=13.0, A=26.9815, rho=2700.0),
    "Cu": dict(Z=29.0, A=63.546, rho=8960.0),
    "Au": dict(Z=79.0, A=196.967, rho=19300.0),
    "Ta": dict(Z=73.0, A=180.948, rho=16650.0),
}

# physics toggle bits (mirrors the HYB_PHYS_* bits of the C ABI)
PHYS_FIELDS = 1 << 0      # gather E and B in the push
PHYS_ION = 1 << 1         # continuous ionisation loss
PHYS_BREM = 1 << 2        # bremsstrahlung (discrete + sub-cut)
PHYS_SCATTER = 1 << 3     # Davies elastic scatter
PHYS_EVOLVE_E = 1 << 4    # recompute E from Ohm's law each step
PHYS_EVOLVE_B = 1 << 5    # advance B with Faraday's law
PHYS_HEAT = 1 << 6        # temperature and resistivity update
PHYS_FSIGMA = 1 << 7       # eq. F_sigma enhancement of the brem cross-sections (opt-in)
PHYS_DELTA = 1 << 8        # delta rays + restricted ionisation loss (opt-in)
PHYS_URBAN = 1 << 9        # Urban-type elastic scatter instead of Davies (opt-in, with PHYS_SCATTER)
PHYS_ALL = (PHYS_FIELDS | PHYS_ION | PHYS_BREM | PHYS_SCATTER |
            PHYS_EVOLVE_E | PHYS_EVOLVE_B | PHYS_HEAT)

FP64 = 0
FP32_MIXED = 1

# boundary kinds per axis (x: the slab faces; y, z: the domain walls)
BC_REFLUX = 0    # escape above kappa_esc a0 m c^2, else reflux (Sec. II.A)
BC_OPEN = 1      # every electron that leaves escapes
BC_MIRROR = 2    # specular reflection, no loss
BC_PERIODIC = 3  # y, z only: leave through one wall, re-enter through the other (no field feedback)

TABLE_CSBH = 0   # complete-screening Bethe-Heitler spectral shape
TABLE_FLAT = 1   # flat k dsigma/dk


def intensity_wcm2(i_wcm2: float) -> float:
    """W/cm^2 -> W/m^2."""
    return i_wcm2 * 1e4


def base_config(**over) -> dict:
    """A run configuration with the paper's defaults (Sec. II.A, II.B)."""
    cfg = dict(
        nx=32, ny=16, nz=16, dx=1e-6, dt=10e-15,
        precision=FP64,
        material="Au",
        I_ex=0.0,                     # 0 -> 11 eV * Z (Sec. III.B)
        x_lo=2e-6, x_hi=30e-6,        # slab x-extent; y and z span the domain
        T0=EV / KB,                   # 1 eV in kelvin
        lambda1=7.0, lambda2=3.5,     # reduced Lee-More fit (App. A)
        I0=intensity_wcm2(1e20), wavelength=1e-6,
        kappa_esc=2.0, kappa_tnsa=2.7e-3, sigma_dtheta=math.radians(23.0),
        reflux_ke_frac=0.0,           # 0 -> paper momentum-loss mode
        brem_boost=1.0, k_cut=1e3 * EV,
        table_shape=TABLE_CSBH, table_nT=128, table_nr=256, table_emax=10e9 * EV,
        e_min=10e3 * EV,
        delta_cut=1e3 * EV,           # delta-ray cut (App. B: 1 keV)
        tally_nE=16, tally_ntheta=32, tally_Elo=10e3 * EV, tally_Ehi=1e9 * EV,
        tally_Ethr=1.0 * MEV,
        series_len=256,
        seed=0,
        max_particles=1 << 16,
        physics=PHYS_ALL,
        eta_fixed=0.0,
        n_sub=0,                      # 0 -> automatic from the stability scan
        sort_every=0,
        bc_x=BC_REFLUX, bc_y=BC_REFLUX, bc_z=BC_REFLUX,
        # further elements mixed into the slab (App. A compounds): Z, molar
        # mass [g/mol], partial mass density [kg/m^3], I_ex [J] (0 -> 11 eV Z)
        n_extra=0, extra_Z=(0.0, 0.0, 0.0), extra_A=(0.0, 0.0, 0.0), extra_rho=(0.0, 0.0, 0.0),
        extra_I_ex=(0.0, 0.0, 0.0),
    )
    for k, v in over.items():
        if k not in cfg and k not in ("Z", "A", "rho"):
            raise KeyError(f"unknown config key {k}")
        cfg[k] = v
    mat = MATERIALS[cfg["material"]]
    cfg.setdefault("Z", mat["Z"])
    cfg.setdefault("A", mat["A"])
    cfg.setdefault("rho", mat["rho"])
    return cfg


def source(**over) -> dict:
    """One injection source: exponential energies, Gaussian spot, uniform cone."""
    src = dict(
        n_macro=10000, t_start=0.0, t_end=1e-12,
        y0=8e-6, z0=8e-6, r_fwhm=5e-6,
        T_hot=0.86 * MEV, half_angle=math.radians(30.0),
        eta_l2e=0.3, weight=0.0,       # 0 -> weight from I0 and eta_l2e
    )
    for k, v in over.items():
        if k not in src:
            raise KeyError(f"unknown source key {k}")
        src[k] = v
    return src


def config_small() -> tuple[dict, list[dict], int]:
    """Plain FP64 gold slab, 32x16x16 cells of 1 um, 1e4 macro-electrons,
    200 steps of 10 fs, 1 % kinetic-energy loss per reflux, 16x32 tally.
    Returns (config, sources, steps)."""
    cfg = base_config(
        nx=32, ny=16, nz=16, dx=1e-6, dt=10e-15, precision=FP64,
        material="Au", x_lo=2e-6, x_hi=30e-6,
        I0=intensity_wcm2(1e20), reflux_ke_frac=0.01,
        tally_nE=16, tally_ntheta=32, series_len=256,
        max_particles=1 << 14, seed=0)
    src = source(n_macro=10000, t_start=0.0, t_end=1e-12, y0=8e-6, z0=8e-6,
                 r_fwhm=5e-6, T_hot=0.86 * MEV, half_angle=math.radians(30.0))
    return cfg, [src], 200


def config_fp64_large() -> tuple[dict, list[dict], int]:
    """FP64 gold slab 200 um thick in a 256x128x128 grid of 1 um cells,
    2e7 macro-electrons at T_hot = 3.4 MeV (1e21 W/cm^2), 3 um spot,
    40 deg cone, 20 fs steps, 2000 steps, paper reflux, 64x90 tally."""
    cfg = base_config(
        nx=256, ny=128, nz=128, dx=1e-6, dt=20e-15, precision=FP64,
        material="Au", x_lo=2e-6, x_hi=202e-6,
        I0=intensity_wcm2(1e21), reflux_ke_frac=0.0,
        tally_nE=64, tally_ntheta=90, series_len=2048,
        max_particles=20_000_000, seed=0, sort_every=1)
    src = source(n_macro=20_000_000, t_start=0.0, t_end=1e-12, y0=64e-6,
                 z0=64e-6, r_fwhm=3e-6, T_hot=3.4 * MEV,
                 half_angle=math.radians(40.0))
    return cfg, [src], 2000


def config_mixed_large() -> tuple[dict, list[dict], int]:
    """FP32-mixed gold slab x in [2, 254] um of a 256^3 grid, 1e8
    macro-electrons at T_hot = 10.8 MeV (1e22 W/cm^2), 5 um spot, 30 deg
    cone, 1 % reflux loss, 5000 steps of 20 fs, 64x90 tally."""
    cfg = base_config(
        nx=256, ny=256, nz=256, dx=1e-6, dt=20e-15, precision=FP32_MIXED,
        material="Au", x_lo=2e-6, x_hi=254e-6,
        I0=intensity_wcm2(1e22), reflux_ke_frac=0.01,
        tally_nE=64, tally_ntheta=90, series_len=5000,
        max_particles=100_000_000, seed=0, sort_every=1)
    src = source(n_macro=100_000_000, t_start=0.0, t_end=1e-12, y0=128e-6,
                 z0=128e-6, r_fwhm=5e-6, T_hot=10.8 * MEV,
                 half_angle=math.radians(30.0))
    return cfg, [src], 5000


def config_huge() -> tuple[dict, list[dict], int]:
    """FP32-mixed 512^3 grid of 0.5 um cells, gold 250 um thick, 2e8
    macro-electrons at 10.8 MeV, 2 um spot, 10000 steps of 10 fs, 128x180."""
    cfg = base_config(
        nx=512, ny=512, nz=512, dx=0.5e-6, dt=10e-15, precision=FP32_MIXED,
        material="Au", x_lo=2e-6, x_hi=252e-6,
        I0=intensity_wcm2(1e22), reflux_ke_frac=0.0,
        tally_nE=128, tally_ntheta=180, series_len=10000,
        max_particles=200_000_000, seed=0, sort_every=1)
    src = source(n_macro=200_000_000, t_start=0.0, t_end=1e-12, y0=128e-6,
                 z0=128e-6, r_fwhm=2e-6, T_hot=10.8 * MEV,
                 half_angle=math.radians(30.0))
    return cfg, [src], 10000


def plastic(**over) -> dict:
    """A CH plastic slab (polystyrene-like, 1.05 g/cm^3, C:H = 1:1) as a
    compound of carbon (the first element) and hydrogen: the config keys of
    base_config for it."""
    n = 1050.0 / ((12.011 + 1.008) * 1.66053906660e-27)     # CH units per m^3
    rho_c = n * 12.011 * 1.66053906660e-27
    rho_h = n * 1.008 * 1.66053906660e-27
    cfg = dict(material="Au", Z=6.0, A=12.011, rho=rho_c, n_extra=1, extra_Z=(1.0, 0.0, 0.0),
               extra_A=(1.008, 0.0, 0.0), extra_rho=(rho_h, 0.0, 0.0), extra_I_ex=(0.0, 0.0, 0.0))
    cfg.update(over)
    return cfg


def beam(**over) -> dict:
    """A mono-energetic beam at normal incidence: per_cell macro-electrons of
    the given weight in every face cell of the slab's front, at the step of
    t_start."""
    b = dict(per_cell=50, t_start=0.0, energy=0.5 * MEV, weight=1.0)
    for k, v in over.items():
        if k not in b:
            raise KeyError(f"unknown beam key {k}")
        b[k] = v
    return b


def config_depth_dose(urban: bool = False) -> tuple[dict, dict, int]:
    """The paper's depth-dose benchmark setup (App. C): 0.5 MeV electrons at
    normal incidence on tantalum, 256 x 8 x 8 cells over 150 um in x, 50
    unit-weight macro-electrons per front-face cell in the first step, 2 ps;
    open in x, periodic in y and z as in the paper; ionisation, Davies scatter and
    heating (currents of unit-weight electrons give negligible fields).
    Cells are cubic here (150/256 um), so the lateral extent is 4.7 um.
    urban: the paper's other elastic model (Urban-type model functions)
    instead of Davies.  Returns (config, beam, steps)."""
    nx = 256
    dx = 150e-6 / nx
    cfg = base_config(nx=nx, ny=8, nz=8, dx=dx, dt=5e-15, material="Ta", x_lo=0.0, x_hi=nx * dx,
                      physics=PHYS_ION | PHYS_SCATTER | PHYS_HEAT | (PHYS_URBAN if urban else 0),
                      bc_x=BC_OPEN, bc_y=BC_PERIODIC,
                      bc_z=BC_PERIODIC, max_particles=4096, series_len=4)
    return cfg, beam(), 400


def model_inputs(**over) -> dict:
    """Inputs of the paper's energy-partition model (Sec. III.B): 100 um
    cube, 5 um / 40 fs envelope with <fg> 0.41 and <sqrt fg> 0.61,
    eta_l->e 0.3, kappa_esc 2, kappa_tnsa 2.7e-3, 1 MeV threshold, current
    cone 20 deg, <eta> 1e-6 Ohm m, n_i 6e28 m^-3, 1 um light; 4000
    integration steps per macro-electron."""
    m = dict(wavelength=1e-6, eta_l2e=0.3, r_fwhm=5e-6, t_fwhm=40e-15, fg_mean=0.41, sqrt_fg_mean=0.61,
             kappa_esc=2.0, kappa_tnsa=2.7e-3, e_th=1.0 * MEV, Lx=100e-6, Ly=100e-6, Lz=100e-6,
             theta_c=math.radians(20.0), eta_mean=1e-6, n_i=6e28, nsteps=4000)
    for k, v in over.items():
        if k not in m:
            raise KeyError(f"unknown model key {k}")
        m[k] = v
    return m


def model_scan_grid(n_int: int = 41, z_values=None) -> tuple[np.ndarray, np.ndarray]:
    """The intensity-Z plane of the model's heatmap: n_int log-spaced
    intensities over 1e20-1e22 W/cm^2 (in W/m^2) times atomic numbers
    (default 1..92); returns flat (I0, Z) arrays."""
    z = np.arange(1, 93, dtype=np.float64) if z_values is None else np.asarray(z_values, dtype=np.float64)
    i0 = intensity_wcm2(np.logspace(20.0, 22.0, n_int))
    I, Z = np.meshgrid(i0, z, indexing="ij")
    return I.ravel(), Z.ravel()


def scale_particles(cfg: dict, srcs: list[dict], n_macro: int) -> tuple[dict, list[dict]]:
    """Same workload with fewer macro-electrons (same physics per electron:
    the default weight rule keeps the injected energy fixed)."""
    cfg = copy.deepcopy(cfg)
    srcs = copy.deepcopy(srcs)
    tot = sum(s["n_macro"] for s in srcs)
    for s in srcs:
        s["n_macro"] = max(1, int(round(s["n_macro"] * n_macro / tot)))
    cfg["max_particles"] = max(1024, sum(s["n_macro"] for s in srcs))
    return cfg, srcs


# Hot-electron temperatures quoted for 1e20, 1e21 and 1e22 W/cm^2.
_THOT_ANCHORS = [(1e20, 0.86), (1e21, 3.4), (1e22, 10.8)]


def t_hot_mev(i_wcm2: float) -> float:
    """Piecewise power law in log-log through the three anchors above."""
    pts = _THOT_ANCHORS
    li = math.log10(i_wcm2)
    for (i0, t0), (i1, t1) in zip(pts[:-1], pts[1:]):
        if li <= math.log10(i1) or (i1, t1) == pts[-1]:
            f = (li - math.log10(i0)) / (math.log10(i1) - math.log10(i0))
            return 10 ** (math.log10(t0) + f * (math.log10(t1) - math.log10(t0)))
    raise AssertionError


def scan_runs(n_runs: int = 64, seed: int = 0, rate_hz: float = 2.0,
              scale: float = 1.0) -> list[dict]:
    """The parameter-scan request stream: Poisson arrivals (mean rate_hz),
    thickness from {5,20,50,100,200,500} um, Z from {Al, Cu, Au}, intensity
    log-uniform in [1e20, 1e22] W/cm^2, macro-electrons log-uniform in
    [1e5, 1e7] and 500-3000 steps.  `scale` shrinks particle counts and step
    counts for tests.  Returns a list of dicts with keys
    arrival, cfg, srcs, steps."""
    rng = np.random.default_rng(seed)
    thick_um = [5, 20, 50, 100, 200, 500]
    mats = ["Al", "Cu", "Au"]
    t = 0.0
    runs = []
    for r in range(n_runs):
        t += rng.exponential(1.0 / rate_hz)
        th = float(rng.choice(thick_um))
        mat = str(rng.choice(mats))
        i_wcm2 = 10 ** rng.uniform(20.0, 22.0)
        n_macro = int(10 ** rng.uniform(5.0, 7.0) * scale)
        n_macro = max(n_macro, 256)
        steps = int(rng.integers(500, 3001) * scale)
        steps = max(steps, 10)
        # grid: x spans the slab plus 2 um of vacuum on each side
        length = th + 4.0
        nx = 64
        while nx * 1.0 < length and nx < 256:
            nx *= 2
        dx_um = 1.0 if nx * 1.0 >= length else length / 256.0
        # keep the slab aligned with cell faces: x_lo = 2 cells
        ix_lo = 2
        ix_hi = ix_lo + int(round(th / dx_um))
        if ix_hi > nx - 2:
            ix_hi = nx - 2
        ny = nz = nx // 2
        cfg = base_config(
            nx=nx, ny=ny, nz=nz, dx=dx_um * 1e-6, dt=10e-15,
            precision=FP32_MIXED, material=mat,
            x_lo=ix_lo * dx_um * 1e-6, x_hi=ix_hi * dx_um * 1e-6,
            I0=intensity_wcm2(i_wcm2), reflux_ke_frac=0.0,
            tally_nE=64, tally_ntheta=90, series_len=max(steps, 1),
            max_particles=n_macro, seed=r, sort_every=1)
        half = ny * dx_um * 1e-6 / 2
        src = source(n_macro=n_macro, t_start=0.0, t_end=1e-12, y0=half,
                     z0=half, r_fwhm=min(5e-6, 0.8 * half),
                     T_hot=t_hot_mev(i_wcm2) * MEV,
                     half_angle=math.radians(30.0))
        runs.append(dict(arrival=t, cfg=cfg, srcs=[src], steps=steps,
                         intensity_wcm2=i_wcm2, thickness_um=th))
    return runs
