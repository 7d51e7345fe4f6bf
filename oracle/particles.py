"""Hot macro-electron physics of the hybrid-PIC step (Sec. II and App. B of
the paper).  Oracle-only implementation: FP64, SI (positions in m, momenta
in kg m/s, energies in J), vectorised over particles with NumPy.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as K
from . import philox as P

Q_E = -K.E            # electron charge


# --------------------------------------------------------------------------
# kinematics
# --------------------------------------------------------------------------
def gamma_of(p):
    """Lorentz factor of momenta p (n, 3)."""
    return np.sqrt(1.0 + np.sum(p * p, axis=-1) / (K.ME * K.C) ** 2)


def kinetic(p):
    """Kinetic energy (gamma - 1) m c^2 written as p^2 / ((gamma + 1) m),
    which has no cancellation at low energy."""
    return np.sum(p * p, axis=-1) / ((gamma_of(p) + 1.0) * K.ME)


def momentum_of_energy(eps):
    """|p| of an electron of kinetic energy eps: p c = sqrt(eps (eps + 2 m c^2))."""
    return np.sqrt(eps * (eps + 2.0 * K.MEC2)) / K.C


def with_energy(p, eps):
    """Rescale momenta p to kinetic energies eps keeping their directions."""
    pm = np.sqrt(np.sum(p * p, axis=-1))
    scale = np.where(pm > 0.0, momentum_of_energy(np.maximum(eps, 0.0)) / np.where(pm > 0, pm, 1.0), 0.0)
    return p * scale[:, None]


def a0_of(I0, wavelength):
    """Normalised vector potential, eq. (a0): a0 = 8.5e-6 sqrt(I0 lambda^2), SI."""
    return 8.5e-6 * math.sqrt(I0 * wavelength * wavelength)


# --------------------------------------------------------------------------
# Yee-staggered linear weighting (gather and deposit share it)
# --------------------------------------------------------------------------
def _axis(X, n, staggered):
    """Indices, signs and weights along one axis for a position X in cell
    units: (i0, i1, f, s0, s1) with weight 1-f on i0 and f on i1.  Node
    quantities sit at integers, staggered ones at half-integers.  A staggered
    index one past either end is a mirror ghost: it maps to the nearest valid
    index with sign -1 (odd about the wall)."""
    Xs = X - 0.5 if staggered else X
    i0 = np.floor(Xs).astype(np.int64)
    f = Xs - i0
    i1 = i0 + 1
    s0 = np.ones_like(f)
    s1 = np.ones_like(f)
    if staggered:
        s0 = np.where(i0 < 0, -1.0, 1.0)
        s1 = np.where(i1 > n - 1, -1.0, 1.0)
        i0 = np.clip(i0, 0, n - 1)
        i1 = np.clip(i1, 0, n - 1)
    return i0, i1, f, s0, s1


# staggering (x, y, z) of the six field components and of j_h
STAG_E = ((True, False, False), (False, True, False), (False, False, True))
STAG_B = ((False, True, True), (True, False, True), (True, True, False))


def stencil(X, dims, stag):
    """Per-component stencil for positions X in cell units (x / dx): a list
    over components of three axis tuples."""
    return [[_axis(X[:, d], dims[d], s[d]) for d in range(3)] for s in stag]


def _corners(st):
    """The 8 (index, weight) corners of one component's stencil."""
    (ix0, ix1, fx, sx0, sx1), (iy0, iy1, fy, sy0, sy1), (iz0, iz1, fz, sz0, sz1) = st
    for ix, wx in ((ix0, sx0 * (1.0 - fx)), (ix1, sx1 * fx)):
        for iy, wy in ((iy0, sy0 * (1.0 - fy)), (iy1, sy1 * fy)):
            for iz, wz in ((iz0, sz0 * (1.0 - fz)), (iz1, sz1 * fz)):
                yield (ix, iy, iz), wx * wy * wz


def interp(F, st):
    """Trilinear interpolation of one component array with stencil st."""
    v = 0.0
    for idx, wgt in _corners(st):
        v = v + wgt * F[idx]
    return v


def gather(X, E, B, dims):
    """E and B at particle positions X (cell units), (n, 3) each."""
    se = stencil(X, dims, STAG_E)
    sb = stencil(X, dims, STAG_B)
    Ep = np.stack([interp(E[c], se[c]) for c in range(3)], axis=-1)
    Bp = np.stack([interp(B[c], sb[c]) for c in range(3)], axis=-1)
    return Ep, Bp


def deposit(j, X, vel, w, dx, dims):
    """j_h += q w v S(x) / dx^3 on the E positions with the gather's weights
    (a ghost's share goes to its mirror index with the ghost's sign).
    X in cell units."""
    se = stencil(X, dims, STAG_E)
    amp = Q_E * w / dx ** 3
    for c in range(3):
        for idx, wgt in _corners(se[c]):
            np.add.at(j[c], idx, amp * vel[:, c] * wgt)


# --------------------------------------------------------------------------
# Boris push (q = -e)
# --------------------------------------------------------------------------
def boris(p, Ep, Bp, dt):
    """Relativistic Boris rotation: half electric kick, magnetic rotation with
    t = q B dt / (2 gamma m), s = 2 t / (1 + t^2), half electric kick."""
    pm = p + 0.5 * Q_E * dt * Ep
    g = gamma_of(pm)
    t = (0.5 * Q_E * dt / (g * K.ME))[:, None] * Bp
    s = 2.0 * t / (1.0 + np.sum(t * t, axis=-1))[:, None]
    pp = pm + np.cross(pm, t)
    pplus = pm + np.cross(pp, s)
    return pplus + 0.5 * Q_E * dt * Ep


# --------------------------------------------------------------------------
# rotations about the momentum direction
# --------------------------------------------------------------------------
def rotate(p, dtheta, phi):
    """Turn the directions of p by polar angle dtheta at azimuth phi, keeping
    |p|.  Basis: a = unit(phat x e_m), with e_m the axis of the smallest
    |phat_i| (ties -> lowest index), b = phat x a;
    phat' = cos(dtheta) phat + sin(dtheta) (cos(phi) a + sin(phi) b)."""
    pm = np.sqrt(np.sum(p * p, axis=-1))
    ph = p / pm[:, None]
    m = np.argmin(np.abs(ph), axis=-1)
    em = np.zeros_like(ph)
    em[np.arange(len(m)), m] = 1.0
    a = np.cross(ph, em)
    a /= np.sqrt(np.sum(a * a, axis=-1))[:, None]
    b = np.cross(ph, a)
    d = (np.cos(dtheta)[:, None] * ph
         + np.sin(dtheta)[:, None] * (np.cos(phi)[:, None] * a + np.sin(phi)[:, None] * b))
    d /= np.sqrt(np.sum(d * d, axis=-1))[:, None]
    return d * pm[:, None]


# --------------------------------------------------------------------------
# collisions
# --------------------------------------------------------------------------
def stopping_ion(eps, p, Z, n_i, I_ex):
    """Continuous ionisation stopping power eq. (stop_ion) [J/m], clamped >= 0:
    Z n_i e^4/(4 pi eps0^2 m v^2) (ln(eps/I) + ln(gamma+1)/2 + 0.909/gamma^2
    - 0.818/gamma - 0.246)."""
    g = gamma_of(p)
    v2 = np.sum(p * p, axis=-1) / (g * K.ME) ** 2
    L = (np.log(np.maximum(eps, 1e-300) / I_ex) + 0.5 * np.log(g + 1.0)
         + 0.909 / g ** 2 - 0.818 / g - 0.246)
    S = Z * n_i * K.E ** 4 / (4.0 * math.pi * K.EPS0 ** 2 * K.ME * v2) * L
    return np.maximum(S, 0.0)


def stopping_ion_mix(eps, p, elems):
    """eq. (stop_ion) summed over the elements of a compound (App. A), each
    with its own Z, n and I_ex; the total clamped >= 0."""
    g = gamma_of(p)
    v2 = np.sum(p * p, axis=-1) / (g * K.ME) ** 2
    common = 0.5 * np.log(g + 1.0) + 0.909 / g ** 2 - 0.818 / g - 0.246
    S = 0.0
    for e in elems:
        L = np.log(np.maximum(eps, 1e-300) / e["I_ex"]) + common
        S = S + e["Z"] * e["n"] * K.E ** 4 / (4.0 * math.pi * K.EPS0 ** 2 * K.ME * v2) * L
    return np.maximum(S, 0.0)


def davies_sigma2_mix(p, elems, dt):
    """The Davies variance summed over the elements of a compound (each
    Z^2 n with its own screening logarithm), the total clamped >= 0."""
    g = gamma_of(p)
    pm = np.sqrt(np.sum(p * p, axis=-1))
    s = 0.0
    for e in elems:
        lg = np.log(4.0 * K.EPS0 * K.H * pm / (e["Z"] ** (1.0 / 3.0) * K.ME * K.E ** 2))
        s = s + e["Z"] * e["Z"] * e["n"] * lg
    return (K.E ** 4 * g * K.ME / (2.0 * math.pi * K.EPS0 ** 2 * pm ** 3) * np.maximum(s, 0.0) * dt)


def davies_sigma2(p, Z, n_i, dt):
    """Variance of the Davies deflection over dt (App. B):
    Z^2 e^4 n_i gamma m/(2 pi eps0^2 p^3) ln(4 eps0 h p/(Z^1/3 m e^2)) dt,
    logarithm clamped at zero."""
    g = gamma_of(p)
    pm = np.sqrt(np.sum(p * p, axis=-1))
    lg = np.log(4.0 * K.EPS0 * K.H * pm / (Z ** (1.0 / 3.0) * K.ME * K.E ** 2))
    return (Z * Z * K.E ** 4 * n_i * g * K.ME / (2.0 * math.pi * K.EPS0 ** 2 * pm ** 3)
            * np.maximum(lg, 0.0) * dt)


def box_muller(u0, u1):
    """Standard normal deviate from two uniforms."""
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * math.pi * u1)


TSAI_A = 0.625      # rate of the first Gamma(2) component of the Tsai-based mixture
TSAI_D = 27.0       # relative weight of the second component (rate 3 TSAI_A)


def photon_polar(gamma, r, r2):
    """Photon polar angle about the electron direction (App. B: a direction
    drawn from the Tsai differential cross-section).  The published
    approximation of the Tsai angular distribution: theta = u / gamma with u
    of density proportional to u exp(-a u) + d u exp(-3 a u), a = 0.625,
    d = 27 -- a mixture of Gamma(2) laws of rates a (weight 9/(9+d)) and 3a
    (weight d/(9+d)), each drawn as -ln(r1 r2)/rate.  The uniform r picks the
    component and, rescaled onto (0, 1), serves as r1; theta is capped at pi."""
    p1 = 9.0 / (9.0 + TSAI_D)
    first = r < p1
    r1 = np.where(first, r / p1, (r - p1) / (1.0 - p1))
    rate = np.where(first, TSAI_A, 3.0 * TSAI_A)
    return np.minimum(-np.log(r1 * r2) / rate / gamma, math.pi)


# --------------------------------------------------------------------------
# injection (App. B: exponential spectrum; Sec. II.B: Gaussian spot, cone)
# --------------------------------------------------------------------------
def injection_schedule(src, dt):
    """(first step, number of steps) of a source: uniform count per step over
    [t_start, t_end), the remainder going to the earliest steps."""
    s0 = int(math.floor(src["t_start"] / dt + 0.5))
    ns = max(1, int(math.floor((src["t_end"] - src["t_start"]) / dt + 0.5)))
    return s0, ns


def default_weight(src, I0):
    """Real electrons per macro-electron: the injected hot-electron energy
    I0 <f> (pi r_fwhm^2/4) tau eta_l2e (eq. N_cell summed over the spot with a
    flat time envelope) divided by N_macro T_hot.  <f> = 1/(2 ln 2) is the
    mean of f = 2^-(2r/r_fwhm)^2 over the disc f >= 1/2."""
    if src["weight"] > 0.0:
        return src["weight"]
    f_mean = 1.0 / (2.0 * math.log(2.0))
    tau = src["t_end"] - src["t_start"]
    energy = I0 * f_mean * (math.pi * src["r_fwhm"] ** 2 / 4.0) * tau * src["eta_l2e"]
    return energy / (src["n_macro"] * src["T_hot"])


def inject(src, first_id, count, step, seed, ix_lo, dx, I0):
    """`count` macro-electrons with ids first_id.. at step `step`.
      radius: r^2 = -2 s^2 ln(1 - u/2), s^2 = r_fwhm^2/(8 ln 2)  (f >= 1/2 disc)
      energy: eps = -T_hot ln(1 - u)
      direction: cos(theta) = 1 - u (1 - cos(theta_max)), phi = 2 pi u, about +x
      optical depth: tau = -ln(1 - u)
    Positions are returned in cell units (x / dx); the slab front face is the
    integer ix_lo.  Returns X, p, w, tau, ids."""
    ids = (np.arange(count, dtype=np.uint64) + np.uint64(first_id)).astype(np.uint64)
    a0, a1, a2, a3 = P.uniforms(ids, seed, step, P.SLOT_INJECT_A)
    b0, b1, _, _ = P.uniforms(ids, seed, step, P.SLOT_INJECT_B)
    s2 = src["r_fwhm"] ** 2 / (8.0 * math.log(2.0))
    r = np.sqrt(-2.0 * s2 * np.log(1.0 - 0.5 * a0))
    ps = 2.0 * math.pi * a1
    pos = np.stack([np.full(count, float(ix_lo)), (src["y0"] + r * np.cos(ps)) / dx,
                    (src["z0"] + r * np.sin(ps)) / dx], axis=-1)
    eps = -src["T_hot"] * np.log(1.0 - a2)
    ct = 1.0 - a3 * (1.0 - math.cos(src["half_angle"]))
    st = np.sqrt(np.maximum(1.0 - ct * ct, 0.0))
    pc = 2.0 * math.pi * b0
    d = np.stack([ct, st * np.cos(pc), st * np.sin(pc)], axis=-1)
    p = d * momentum_of_energy(eps)[:, None]
    tau = -np.log(1.0 - b1)
    w = np.full(count, default_weight(src, I0))
    return pos, p, w, tau, ids.astype(np.uint32)


def inject_beam(beam, first_id, step, seed, ix_lo, ny, nz):
    """A mono-energetic beam at normal incidence: per_cell electrons in each
    face cell (j, k) of the slab's front, k-major, uniform over the cell's
    face; kinetic energy `energy`, momentum along +x, weight `weight`,
    optical depth -ln(1 - u).  Returns X (cell units), p, w, tau, ids."""
    per = int(beam["per_cell"])
    n = per * ny * nz
    ids = (np.arange(n, dtype=np.uint64) + np.uint64(first_id)).astype(np.uint64)
    a0_, a1, _, _ = P.uniforms(ids, seed, step, P.SLOT_INJECT_A)
    _, b1, _, _ = P.uniforms(ids, seed, step, P.SLOT_INJECT_B)
    cell = np.arange(n) // per
    jj, kk = (cell % ny).astype(np.float64), (cell // ny).astype(np.float64)
    pos = np.stack([np.full(n, float(ix_lo)), jj + a0_, kk + a1], axis=-1)
    p = np.zeros((n, 3))
    p[:, 0] = momentum_of_energy(np.full(n, float(beam["energy"])))
    tau = -np.log(1.0 - b1)
    w = np.full(n, float(beam["weight"]))
    return pos, p, w, tau, ids.astype(np.uint32)


# ---------------------------------------------------------------------------
# the paper's injection envelope (Sec. II.B, eq. N_cell, App. B)
# ---------------------------------------------------------------------------
def envelope_cells(env, ny, nz, dx):
    """Face cells (j, k) that inject, in k-major order, with their f:
    f = 2^-(2r/r_fwhm)^2 at the cell centre, kept where f >= f_min."""
    out = []
    for k in range(nz):
        for j in range(ny):
            r = math.hypot((j + 0.5) * dx - env["y0"], (k + 0.5) * dx - env["z0"])
            f = 2.0 ** (-(2.0 * r / env["r_fwhm"]) ** 2)
            if f >= env["f_min"]:
                out.append((j, k, f))
    return out


def envelope_g(env, step, dt):
    """Temporal envelope at the middle of step `step`: 2^-(2(t - t_peak)/t_fwhm)^2."""
    t = (step + 0.5) * dt
    return 2.0 ** (-(2.0 * (t - env["t_peak"]) / env["t_fwhm"]) ** 2)


def envelope_steps(env, dt):
    """(first step, number of steps) with g >= g_min; g is unimodal, so they
    are contiguous."""
    half = 0.5 * env["t_fwhm"] * math.sqrt(math.log2(1.0 / env["g_min"]))
    lo = max(0, int(math.floor((env["t_peak"] - half) / dt)) - 2)
    steps = [n for n in range(lo, lo + int((2 * half) / dt) + 6) if envelope_g(env, n, dt) >= env["g_min"]]
    return steps[0], len(steps)


def envelope_weight_max(env, I0, a0, dx, dt):
    """Real electrons per macro-electron where f = g = 1: eq. N_cell with
    <eps_k> = a0 m c^2, transverse cell area dx^2, divided by per_cell.  A cell
    of envelope fg carries this times sqrt(fg) (its mean energy is
    a0 sqrt(fg) m c^2)."""
    return I0 * dx * dx * dt * env["eta_l2e"] / (a0 * K.MEC2 * env["per_cell"])


def inject_envelope(env, cells, first_id, step, seed, ix_lo, dx, dt, I0, a0):
    """per_cell macro-electrons in each injecting face cell at step `step`,
    ids first_id.. in (cell, electron) order:
      position: uniform over the cell's face on the slab front
      energy: exponential with mean a m c^2, a = a0 sqrt(f g)
      direction: uniform in a cone about +x of half-angle
                 min(cap, atan(sqrt(2/(gamma - 1)))) (Moore scaling)
      optical depth: tau = -ln(1 - u)
    Returns X (cell units), p, w, tau, ids."""
    per = int(env["per_cell"])
    n = per * len(cells)
    ids = (np.arange(n, dtype=np.uint64) + np.uint64(first_id)).astype(np.uint64)
    a0_, a1, a2, a3 = P.uniforms(ids, seed, step, P.SLOT_INJECT_A)
    b0, b1, _, _ = P.uniforms(ids, seed, step, P.SLOT_INJECT_B)
    jj = np.repeat(np.array([c[0] for c in cells], dtype=np.float64), per)
    kk = np.repeat(np.array([c[1] for c in cells], dtype=np.float64), per)
    f = np.repeat(np.array([c[2] for c in cells]), per)
    g = envelope_g(env, step, dt)
    sq = np.sqrt(f * g)
    pos = np.stack([np.full(n, float(ix_lo)), jj + a0_, kk + a1], axis=-1)
    eps = -(a0 * sq * K.MEC2) * np.log(1.0 - a2)
    gm1 = eps / K.MEC2
    th_max = np.minimum(env["max_half_angle"], np.arctan(np.sqrt(2.0 / gm1)))
    ct = 1.0 - a3 * (1.0 - np.cos(th_max))
    st = np.sqrt(np.maximum(1.0 - ct * ct, 0.0))
    pc = 2.0 * math.pi * b0
    d = np.stack([ct, st * np.cos(pc), st * np.sin(pc)], axis=-1)
    p = d * momentum_of_energy(eps)[:, None]
    tau = -np.log(1.0 - b1)
    w = envelope_weight_max(env, I0, a0, dx, dt) * sq
    return pos, p, w, tau, ids.astype(np.uint32)
