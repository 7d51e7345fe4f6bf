"""One hybrid-PIC run: state, the per-step algorithm, the energy ledger and
the photon tallies.  Oracle-only implementation, FP64, SI.

Per-step order (the paper gives the pieces, not their order; this order is
the reading both implementations follow):
  1. inject the step's scheduled macro-electrons
  2. gather E, B at x^n; Boris push; field work -> ledger
  3. deposit j_h at x^n with the pushed velocity (every particle alive at
     the start of the step)
  4. move x^{n+1} = x^n + v dt
  5. ionisation loss (eq. stop_ion) -> ledger and the cell's heat; with
     delta rays, the restricted loss below the cut instead (App. B)
  5b. delta rays (App. B), optional: Moller scatter above the cut by the
     optical-depth method with a depth of its own, at most one per step;
     the delta ray is born at x^n, below e_min its energy is the cell's heat
  6. bremsstrahlung by the optical-depth method (App. B), at most one
     emission per step, boosted cross-section (Sec. II.B); sub-cut loss;
     optionally both enhanced by eq. F_sigma of the cell at x^n, from the
     temperatures at the start of the step
  7. elastic scatter (App. B): Davies, or Urban-type model functions
     matched to the Lewis moments
  8. boundaries x, y, z: escape or reflux (Sec. II.A); per axis also open
     (every electron leaving escapes), a lossless mirror, or (y, z)
     periodic
  9. removal below e_min, remaining energy -> the cell's heat
 10. n_sub sub-cycles of Ohm + Faraday (App. A)
 11. Ohmic + ionisation heating, electron-ion exchange, resistivity (App. A)
 12. the step's delta rays join the run, ids in (tile of the birth cell,
     parent id) order after those of earlier steps
The heat of a particle goes to the cell that contains x^n.
Positions are held in cell units X = x / dx so that the slab faces and the
walls are exact integers.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as K
from . import fields as F
from . import moller as M
from . import particles as PT
from . import philox as P
from . import solid as S
from . import tables as T
from . import urban as U

PHYS_FIELDS = 1 << 0
PHYS_ION = 1 << 1
PHYS_BREM = 1 << 2
PHYS_SCATTER = 1 << 3
PHYS_EVOLVE_E = 1 << 4
PHYS_EVOLVE_B = 1 << 5
PHYS_HEAT = 1 << 6
PHYS_FSIGMA = 1 << 7
PHYS_DELTA = 1 << 8
PHYS_URBAN = 1 << 9
BC_REFLUX, BC_OPEN, BC_MIRROR, BC_PERIODIC = 0, 1, 2, 3
DELTA_ID_BIT = 0x80000000    # delta rays take ids DELTA_ID_BIT + 0, 1, ...

LEDGER_KEYS = ("injected", "field_loss", "field_gain", "ionisation", "stopped",
               "rad_discrete", "rad_subcut", "escaped", "reflux", "photon_thr", "residual")
COUNTER_KEYS = ("n_injected", "n_emitted", "n_reflux", "n_escaped", "n_stopped", "n_delta",
                "n_delta_lost", "n_electron_steps")


class OracleRun:
    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        c = self.cfg
        self.nx, self.ny, self.nz = int(c["nx"]), int(c["ny"]), int(c["nz"])
        self.dims = (self.nx, self.ny, self.nz)
        self.dx, self.dt = float(c["dx"]), float(c["dt"])
        self.Z, self.A, self.rho = float(c["Z"]), float(c["A"]), float(c["rho"])
        self.n_i = S.ion_density(self.rho, self.A)
        self.I_ex = c["I_ex"] if c["I_ex"] > 0 else 11.0 * K.E * self.Z
        # the solid's elements (App. A: several single-element solids make a
        # compound); the first is (Z, A, rho, I_ex)
        self.elems = [dict(S.element(self.Z, self.A, self.rho), I_ex=self.I_ex)]
        for k in range(int(c.get("n_extra", 0))):
            Zk = float(c["extra_Z"][k])
            Ik = c["extra_I_ex"][k] if c["extra_I_ex"][k] > 0 else 11.0 * K.E * Zk
            self.elems.append(dict(S.element(Zk, c["extra_A"][k], c["extra_rho"][k]), I_ex=Ik))
        if int(c.get("bc_x", BC_REFLUX)) == BC_PERIODIC:
            raise ValueError("the x faces are the slab's: no periodic kind in x")
        if (BC_PERIODIC in (int(c.get("bc_y", 0)), int(c.get("bc_z", 0)))
                and int(c["physics"]) & (PHYS_FIELDS | PHYS_EVOLVE_E | PHYS_EVOLVE_B)):
            raise ValueError("periodic walls are for runs without field feedback")
        if int(c["physics"]) & PHYS_URBAN and not int(c["physics"]) & PHYS_SCATTER:
            raise ValueError("the Urban-type model replaces the Davies scatter: set PHYS_SCATTER too")
        if len(self.elems) > 1 and int(c["physics"]) & PHYS_FSIGMA:
            raise ValueError("eq. F_sigma is defined for single-element solids")
        self.a0 = PT.a0_of(c["I0"], c["wavelength"])
        self.eps_esc = c["kappa_esc"] * self.a0 * K.MEC2
        self.dp_tnsa = c["kappa_tnsa"] * self.a0 * K.ME * K.C
        self.cz = T.c_z(self.Z)
        self.ncz = sum(e["n"] * T.c_z(e["Z"]) for e in self.elems)   # sum of n C_Z
        self.table = T.BremTable(c["k_cut"], c["table_emax"], int(c["table_nT"]),
                                 int(c["table_nr"]), int(c["table_shape"]))
        ix_lo = c["x_lo"] / self.dx
        ix_hi = c["x_hi"] / self.dx
        self.ix_lo, self.ix_hi = int(round(ix_lo)), int(round(ix_hi))
        if abs(ix_lo - self.ix_lo) > 1e-6 or abs(ix_hi - self.ix_hi) > 1e-6:
            raise ValueError("slab faces must lie on cell faces")
        if not (0 <= self.ix_lo < self.ix_hi <= self.nx):
            raise ValueError("slab outside the grid")
        self.box_lo = np.array([float(self.ix_lo), 0.0, 0.0])          # cell units
        self.box_hi = np.array([float(self.ix_hi), float(self.ny), float(self.nz)])
        self.n_sub = int(c["n_sub"]) if c["n_sub"] > 0 else S.n_sub_auto_mix(
            self.dt, self.dx, self.elems, c["T0"], c["lambda1"], c["lambda2"])
        shape = (self.nx + 1, self.ny + 1, self.nz + 1)
        self.E = tuple(np.zeros(shape) for _ in range(3))
        self.B = tuple(np.zeros(shape) for _ in range(3))
        self.j = tuple(np.zeros(shape) for _ in range(3))
        cs = (self.nx, self.ny, self.nz)
        self.solid = np.zeros(cs, dtype=bool)
        self.solid[self.ix_lo:self.ix_hi, :, :] = True
        self.Te = np.full(cs, float(c["T0"]))
        self.Ti = np.full(cs, float(c["T0"]))
        self.eta = np.zeros(cs)
        self.eta[self.solid] = self._eta_of(self.Te[self.solid], self.Ti[self.solid])
        self.ion_heat = np.zeros(cs)
        # particles (kept in id order); X in cell units
        self.X = np.zeros((0, 3))
        self.p = np.zeros((0, 3))
        self.w = np.zeros(0)
        self.tau = np.zeros(0)
        self.taud = np.zeros(0)       # optical depth to the next delta ray
        self.ids = np.zeros(0, dtype=np.uint32)
        self.alive = np.zeros(0, dtype=bool)
        self.step_index = 0
        self.next_id = 0
        self.delta_next = 0
        self.e_cut = float(c.get("delta_cut", 1e3 * K.E))
        self.sources = []
        self.ledger = {k: 0.0 for k in LEDGER_KEYS}
        self.counters = {k: 0 for k in COUNTER_KEYS}
        nE, nth = int(c["tally_nE"]), int(c["tally_ntheta"])
        self.hist_E = np.zeros((nE, nth))
        self.hist_N = np.zeros((nE, nth))
        self.flow = np.zeros(4)       # under E, under N, over E, over N
        self.series = np.zeros(int(c["series_len"]))
        self.last_photons = None

    # ------------------------------------------------------------------
    def _eta_of(self, Te, Ti):
        c = self.cfg
        if c["eta_fixed"] > 0.0:
            return np.full(np.shape(Te), float(c["eta_fixed"]))
        eta, _, _ = S.resistivity_mix(Te, Ti, self.elems, c["lambda1"], c["lambda2"])
        return eta

    def add_source(self, src: dict):
        """Schedule a source; ids are assigned in order of scheduling."""
        s = dict(src)
        s0, ns = PT.injection_schedule(s, self.dt)
        s["_s0"], s["_ns"], s["_id0"] = s0, ns, self.next_id
        s["_w"] = PT.default_weight(s, self.cfg["I0"])
        self.next_id += int(s["n_macro"])
        self.sources.append(s)

    def add_envelope(self, env: dict):
        """Schedule the paper's envelope injection (Sec. II.B): per_cell
        macro-electrons per step in every face cell with f >= f_min, over the
        steps with g >= g_min; ids in (step, cell, electron) order."""
        s = dict(env)
        s["_kind"] = "envelope"
        s["_cells"] = PT.envelope_cells(s, self.ny, self.nz, self.dx)
        s["_s0"], s["_ns"] = PT.envelope_steps(s, self.dt)
        s["_id0"] = self.next_id
        s["_per_step"] = int(s["per_cell"]) * len(s["_cells"])
        self.next_id += s["_per_step"] * s["_ns"]
        self.sources.append(s)

    def add_beam(self, beam: dict):
        """Schedule a mono-energetic beam at normal incidence (the depth-dose
        benchmark of App. C): per_cell electrons in every face cell of the
        slab's front at the step of t_start; ids in (cell k-major, electron)
        order."""
        s = dict(beam)
        s["_kind"] = "beam"
        s["_s0"] = int(math.floor(s["t_start"] / self.dt + 0.5))
        s["_id0"] = self.next_id
        s["_n"] = int(s["per_cell"]) * self.ny * self.nz
        self.next_id += s["_n"]
        self.sources.append(s)

    def _inject(self, n):
        for s in self.sources:
            if s.get("_kind") == "beam":
                if n == s["_s0"]:
                    pos, p, w, tau, ids = PT.inject_beam(s, s["_id0"], n, self.cfg["seed"], self.ix_lo,
                                                         self.ny, self.nz)
                    self._append(pos, p, w, tau, ids, n)
                continue
            if s.get("_kind") == "envelope":
                i = n - s["_s0"]
                if 0 <= i < s["_ns"] and s["_per_step"] > 0:
                    pos, p, w, tau, ids = PT.inject_envelope(
                        s, s["_cells"], s["_id0"] + i * s["_per_step"], n, self.cfg["seed"],
                        self.ix_lo, self.dx, self.dt, self.cfg["I0"], self.a0)
                    self._append(pos, p, w, tau, ids, n)
                continue
            i = n - s["_s0"]
            if i < 0 or i >= s["_ns"]:
                continue
            N, ns = int(s["n_macro"]), s["_ns"]
            base, rem = N // ns, N % ns
            cnt = base + (1 if i < rem else 0)
            if cnt == 0:
                continue
            first = s["_id0"] + i * base + min(i, rem)
            src = dict(s)
            src["weight"] = s["_w"]
            pos, p, w, tau, ids = PT.inject(src, first, cnt, n, self.cfg["seed"],
                                            self.ix_lo, self.dx, self.cfg["I0"])
            self._append(pos, p, w, tau, ids, n)

    def _append(self, pos, p, w, tau, ids, n):
        """Injected electrons; their delta-ray depth is -ln(1 - u) from the
        third draw of the injection's second slot."""
        cnt = len(ids)
        self.ledger["injected"] += float(np.sum(w * PT.kinetic(p)))
        self.counters["n_injected"] += cnt
        taud = np.zeros(cnt)
        if int(self.cfg["physics"]) & PHYS_DELTA:
            taud = -np.log(1.0 - P.uniforms(ids, self.cfg["seed"], n, P.SLOT_INJECT_B)[2])
        self._add(pos, p, w, tau, taud, ids)

    def _add(self, pos, p, w, tau, taud, ids):
        self.X = np.concatenate([self.X, pos])
        self.p = np.concatenate([self.p, p])
        self.w = np.concatenate([self.w, w])
        self.tau = np.concatenate([self.tau, tau])
        self.taud = np.concatenate([self.taud, taud])
        self.ids = np.concatenate([self.ids, ids])
        self.alive = np.concatenate([self.alive, np.ones(len(ids), dtype=bool)])

    def _tally(self, k, wph, dirx, n):
        """Photon tallies: energy (log bins in [E_lo, E_hi)) x angle to +x
        (uniform bins in [0, pi]), energy- and number-weighted."""
        c = self.cfg
        nE, nth = self.hist_E.shape
        th = np.arccos(np.clip(dirx, -1.0, 1.0))
        it = np.minimum(np.floor(nth * th / math.pi).astype(np.int64), nth - 1)
        le = np.log(k / c["tally_Elo"]) / math.log(c["tally_Ehi"] / c["tally_Elo"])
        ie = np.floor(nE * le).astype(np.int64)
        under = ie < 0
        over = ie >= nE
        ok = ~(under | over)
        np.add.at(self.hist_E, (ie[ok], it[ok]), k[ok] * wph[ok])
        np.add.at(self.hist_N, (ie[ok], it[ok]), wph[ok])
        self.flow += [np.sum(k[under] * wph[under]), np.sum(wph[under]),
                      np.sum(k[over] * wph[over]), np.sum(wph[over])]
        thr = k >= c["tally_Ethr"]
        e_thr = float(np.sum(k[thr] * wph[thr]))
        self.ledger["photon_thr"] += e_thr
        if n < len(self.series):
            self.series[n] += e_thr

    # ------------------------------------------------------------------
    def step(self):
        c = self.cfg
        n = self.step_index
        dt, dx = self.dt, self.dx
        phys = int(c["physics"])
        L = self.ledger
        self._inject(n)
        # eq. F_sigma from the temperatures at the start of the step
        fsig = None
        if phys & PHYS_FSIGMA:
            fsig = np.ones_like(self.Te)
            s = self.solid
            fsig[s] = S.f_sigma(self.Te[s], self.Ti[s], self.Z, self.A, self.rho)

        idx = np.nonzero(self.alive)[0]
        pos = self.X[idx].copy()
        p = self.p[idx].copy()
        w = self.w[idx]
        tau = self.tau[idx].copy()
        taud = self.taud[idx].copy()
        ids = self.ids[idx]
        m = len(idx)
        self.counters["n_electron_steps"] += m
        pos_n = pos.copy()             # x^n: birth place of this step's delta rays

        # push
        eps0 = PT.kinetic(p)
        if phys & PHYS_FIELDS:
            Ep, Bp = PT.gather(pos, self.E, self.B, self.dims)
        else:
            Ep = np.zeros((m, 3))
            Bp = np.zeros((m, 3))
        p = PT.boris(p, Ep, Bp, dt)
        eps1 = PT.kinetic(p)
        dW = eps1 - eps0
        L["field_gain"] += float(np.sum(w * np.maximum(dW, 0.0)))
        L["field_loss"] += float(np.sum(w * np.maximum(-dW, 0.0)))
        g1 = PT.gamma_of(p)
        vel = p / (g1 * K.ME)[:, None]

        # deposit (x^n, pushed velocity)
        self.j = tuple(np.zeros_like(a) for a in self.E)
        PT.deposit(self.j, pos, vel, w, dx, self.dims)
        cell = tuple(np.clip(np.floor(pos[:, d]).astype(np.int64), 0, self.dims[d] - 1)
                     for d in range(3))
        self.ion_heat = np.zeros_like(self.Te)

        # move
        pos = pos + vel * (dt / dx)

        # ionisation
        if phys & PHYS_ION:
            if phys & PHYS_DELTA:
                Sion = M.restricted_stopping_mix(eps1, self.elems, self.e_cut)
            else:
                Sion = PT.stopping_ion_mix(eps1, p, self.elems)
            v = np.sqrt(np.sum(vel * vel, axis=-1))
            dE = np.minimum(Sion * v * dt, eps1)
            p = PT.with_energy(p, eps1 - dE)
        eps2 = PT.kinetic(p)
        ion = eps1 - eps2
        L["ionisation"] += float(np.sum(w * ion))
        np.add.at(self.ion_heat, cell, w * ion)

        # delta rays: Moller scatter above the cut, own optical depth
        born = None
        if phys & PHYS_DELTA:
            g2 = PT.gamma_of(p)
            beta = np.sqrt(np.sum(p * p, axis=-1)) / (g2 * K.ME * K.C)
            sig_d = sum(e["n"] * M.moller_sigma(eps2, e["Z"], self.e_cut) for e in self.elems)
            taud = taud - sig_d * beta * K.C * dt
            # no delta ray once eps <= 2 cut (the depth then stays put)
            ie = np.nonzero((taud < 0.0) & (eps2 > 2.0 * self.e_cut))[0]
            if len(ie):
                x = M.sample_fraction(eps2[ie], self.e_cut, M.sampler_uniforms(ids[ie], c["seed"], n))
                e_d = x * eps2[ie]
                uk = P.uniforms(ids[ie], c["seed"], n, P.SLOT_DELTA_K)
                q, d = M.delta_kinematics(p[ie], eps2[ie], e_d, 2.0 * math.pi * uk[0])
                p[ie] = q
                taud[ie] = -np.log(1.0 - uk[1])
                self.counters["n_delta"] += len(ie)
                L["residual"] += float(np.sum(w[ie] * (eps2[ie] - PT.kinetic(q) - e_d)))
                low = e_d < c["e_min"]
                # below e_min the delta ray stops where it is born
                cl = tuple(ci[ie[low]] for ci in cell)
                L["stopped"] += float(np.sum(w[ie[low]] * e_d[low]))
                np.add.at(self.ion_heat, cl, w[ie[low]] * e_d[low])
                k = ~low
                L["residual"] += float(np.sum(w[ie[k]] * (e_d[k] - PT.kinetic(d[k]))))
                born = dict(pos=pos_n[ie[k]], p=d[k], w=w[ie[k]], parent=ids[ie[k]],
                            cell=tuple(ci[ie[k]] for ci in cell))
            eps2 = PT.kinetic(p)

        # bremsstrahlung
        u_c = P.uniforms(ids, c["seed"], n, P.SLOT_COLLIDE)
        kph = np.zeros(m)
        if phys & PHYS_BREM:
            B_ = float(c["brem_boost"])
            g2 = PT.gamma_of(p)
            beta2 = np.sqrt(np.sum(p * p, axis=-1)) / (g2 * K.ME * K.C)
            # cross-sections of the cell at x^n, enhanced by eq. F_sigma if enabled
            fs = fsig[cell] if fsig is not None else 1.0
            tau = tau - B_ * self.ncz * fs * self.table.sigma(eps2) * beta2 * K.C * dt
            emit = tau < 0.0
            sub = self.ncz * fs * self.table.sub(eps2) * beta2 * K.C * dt
            if np.any(emit):
                kph[emit] = self.table.sample_k(eps2[emit], u_c[3][emit])
            p_pre = p.copy()
            sub_a = np.minimum(sub, eps2 - kph / B_)      # sub-cut loss actually applied
            p = PT.with_energy(p, eps2 - kph / B_ - sub_a)
            u_p = P.uniforms(ids, c["seed"], n, P.SLOT_PHOTON)
            tau = np.where(emit, -np.log(1.0 - u_p[2]), tau)
            if np.any(emit):
                th = PT.photon_polar(g2[emit], u_p[0][emit], u_p[3][emit])
                ph = 2.0 * math.pi * u_p[1][emit]
                d = PT.rotate(p_pre[emit], th, ph)
                d = d / np.sqrt(np.sum(d * d, axis=-1))[:, None]
                self._tally(kph[emit], w[emit] / B_, d[:, 0], n)
                self.last_photons = dict(ids=ids[emit], k=kph[emit], w=w[emit] / B_, dir=d)
            else:
                self.last_photons = dict(ids=ids[:0], k=kph[:0], w=w[:0], dir=np.zeros((0, 3)))
            self.counters["n_emitted"] += int(np.sum(emit))
            eps3 = PT.kinetic(p)
            L["rad_discrete"] += float(np.sum(w * kph / B_))
            L["rad_subcut"] += float(np.sum(w * sub_a))
            L["residual"] += float(np.sum(w * ((eps2 - eps3) - kph / B_ - sub_a)))
        else:
            eps3 = eps2

        # elastic scatter: Davies, or the Urban-type model functions
        if phys & PHYS_SCATTER:
            pm = np.sqrt(np.sum(p * p, axis=-1))
            moving = pm > 0.0
            if np.any(moving):
                if phys & PHYS_URBAN:
                    p[moving] = U.scatter(p[moving], self.elems, dt, u_c[0][moving], u_c[1][moving],
                                          u_c[2][moving])
                else:
                    s2 = PT.davies_sigma2_mix(p[moving], self.elems, dt)
                    dth = PT.box_muller(u_c[0][moving], u_c[1][moving]) * np.sqrt(s2)
                    p[moving] = PT.rotate(p[moving], dth, 2.0 * math.pi * u_c[2][moving])
                # elastic: a change of the kinetic energy is rounding, booked apart
                e_r = PT.kinetic(p)
                L["residual"] += float(np.sum(w * (eps3 - e_r)))
                eps3 = e_r
        eps_cur = eps3.copy()

        # boundaries
        alive = np.ones(m, dtype=bool)
        kfrac = float(c["reflux_ke_frac"])
        sig = float(c["sigma_dtheta"])
        for d in range(3):
            lo, hi = self.box_lo[d], self.box_hi[d]
            below = alive & (pos[:, d] < lo)
            above = alive & (pos[:, d] >= hi)
            out = below | above
            if not np.any(out):
                continue
            mode = int(c.get("bc_" + "xyz"[d], BC_REFLUX))
            if mode == BC_PERIODIC:
                # re-enter through the opposite wall, momentum unchanged
                n_d = hi - lo
                x = pos[:, d]
                x = np.where(out, lo + np.mod(x - lo, n_d), x)
                pos[:, d] = np.where(out, np.clip(x, lo, np.nextafter(hi, -np.inf)), x)
                continue
            if mode == BC_MIRROR:
                # specular: mirror the position about the face, flip the normal momentum
                x = pos[:, d]
                x = np.where(below, 2.0 * lo - x, x)
                x = np.where(above, 2.0 * hi - x, x)
                pos[:, d] = np.where(out, np.clip(x, lo, np.nextafter(hi, -np.inf)), x)
                p[out, d] = -p[out, d]
                continue
            esc = out & (eps_cur > self.eps_esc) if mode == BC_REFLUX else out
            L["escaped"] += float(np.sum(w[esc] * eps_cur[esc]))
            self.counters["n_escaped"] += int(np.sum(esc))
            alive &= ~esc
            ref = out & ~esc
            self.counters["n_reflux"] += int(np.sum(ref))
            # mirror about the face, clamp into [lo, hi)
            x = pos[:, d]
            x = np.where(below & ref, 2.0 * lo - x, x)
            x = np.where(above & ref, 2.0 * hi - x, x)
            x = np.where(ref, np.clip(x, lo, np.nextafter(hi, -np.inf)), x)
            pos[:, d] = x
            p[ref, d] = -p[ref, d]
            # momentum or energy loss
            if kfrac > 0.0:
                e_new = eps_cur * (1.0 - kfrac)
                p[ref] = PT.with_energy(p[ref], e_new[ref])
                dead = np.zeros(m, dtype=bool)
            else:
                pm = np.sqrt(np.sum(p * p, axis=-1))
                pm_new = pm - self.dp_tnsa
                dead = ref & (pm_new <= 0.0)
                live = ref & ~dead
                p[live] = p[live] * (pm_new[live] / pm[live])[:, None]
            L["reflux"] += float(np.sum(w[dead] * eps_cur[dead]))
            alive &= ~dead
            live = ref & ~dead
            e_after = PT.kinetic(p[live])
            L["reflux"] += float(np.sum(w[live] * (eps_cur[live] - e_after)))
            eps_cur[live] = e_after
            # scatter by U(-sigma/2, sigma/2) at a uniform azimuth, then point inward
            u_r = P.uniforms(ids, c["seed"], n, P.SLOT_REFLUX[d])
            rot = live & (np.sum(p * p, axis=-1) > 0.0)
            if np.any(rot):
                p[rot] = PT.rotate(p[rot], (u_r[0][rot] - 0.5) * sig,
                                   2.0 * math.pi * u_r[1][rot])
                e_r = PT.kinetic(p[rot])
                L["residual"] += float(np.sum(w[rot] * (eps_cur[rot] - e_r)))
                eps_cur[rot] = e_r
            p[live & below, d] = np.abs(p[live & below, d])
            p[live & above, d] = -np.abs(p[live & above, d])

        # low-energy removal
        stop = alive & (eps_cur < c["e_min"])
        L["stopped"] += float(np.sum(w[stop] * eps_cur[stop]))
        self.counters["n_stopped"] += int(np.sum(stop))
        np.add.at(self.ion_heat, tuple(ci[stop] for ci in cell), w[stop] * eps_cur[stop])
        alive &= ~stop

        self.X[idx] = pos
        self.p[idx] = p
        self.tau[idx] = tau
        self.taud[idx] = taud
        self.alive[idx] = alive

        self.grid_update()
        if born is not None and len(born["w"]):
            self._add_delta_rays(born, n)
        self.step_index += 1

    def grid_update(self):
        """The grid side of the step from this step's hot current self.j and
        collisional heat self.ion_heat: n_sub sub-cycles of Ohm + Faraday
        (App. A, eqs. Ohms_Law, Ampere_Maxwell, Faraday_Lens), then the Ohmic
        and collisional heating, exchange and resistivity of the solid cells
        (App. A, eq. Te_rise)."""
        c = self.cfg
        phys = int(c["physics"])
        dt, dx = self.dt, self.dx
        ev_e = bool(phys & PHYS_EVOLVE_E)
        ev_b = bool(phys & PHYS_EVOLVE_B)
        if ev_e or ev_b:
            self.E, self.B = F.field_update(self.E, self.B, self.j, self.eta, dt, dx,
                                            self.n_sub, ev_e, ev_b)
        if phys & PHYS_HEAT:
            s = self.solid
            j2 = F.cell_current_sq(self.j)
            Te, Ti, eta = S.heat_update_mix(self.Te[s], self.Ti[s], j2[s], self.ion_heat[s],
                                            self.eta[s], dt, dx ** 3, self.elems,
                                            c["lambda1"], c["lambda2"])
            self.Te[s], self.Ti[s] = Te, Ti
            if c["eta_fixed"] <= 0.0:
                self.eta[s] = eta

    def _add_delta_rays(self, born, n):
        """The step's delta rays join the run: ids DELTA_ID_BIT + delta_next +
        rank, ranked by (tile of the birth cell, parent id), tiles of 4^3
        cells numbered x fastest; optical depths -ln(1 - u) from the first
        two draws of the birth slot of the new id."""
        ci, cj, ck = born["cell"]
        ntx, nty = (self.nx + 3) // 4, (self.ny + 3) // 4
        tile = (ci >> 2) + ntx * ((cj >> 2) + nty * (ck >> 2))
        order = np.lexsort((born["parent"].astype(np.int64), tile))
        cnt = len(order)
        if self.delta_next + cnt > DELTA_ID_BIT:
            raise OverflowError("delta-ray ids exhausted")
        ids = (np.uint64(DELTA_ID_BIT + self.delta_next)
               + np.arange(cnt, dtype=np.uint64)).astype(np.uint32)
        u = P.uniforms(ids, self.cfg["seed"], n, P.SLOT_BIRTH)
        self._add(born["pos"][order], born["p"][order], born["w"][order],
                  -np.log(1.0 - u[0]), -np.log(1.0 - u[1]), ids)
        self.delta_next += cnt

    def run(self, nsteps: int):
        for _ in range(nsteps):
            self.step()

    # ------------------------------------------------------------------
    def kinetic_total(self):
        a = self.alive
        return float(np.sum(self.w[a] * PT.kinetic(self.p[a])))

    def closure(self):
        """|injected - (kinetic + losses - gains)| / injected."""
        L = self.ledger
        out = (self.kinetic_total() + L["field_loss"] - L["field_gain"] + L["ionisation"]
               + L["stopped"] + L["rad_discrete"] + L["rad_subcut"] + L["escaped"] + L["reflux"]
               + L["residual"])
        return abs(L["injected"] - out) / max(L["injected"], 1e-300)

    def conversion_efficiency(self):
        """Photon energy above the threshold over injected kinetic energy (eta_e->gamma)."""
        return self.ledger["photon_thr"] / max(self.ledger["injected"], 1e-300)

    @property
    def pos(self):
        """Positions in metres."""
        return self.X * self.dx

    def state(self):
        """Alive particles (in id order, positions in metres), fields, temperatures."""
        a = self.alive
        return dict(pos=self.X[a] * self.dx, p=self.p[a].copy(), w=self.w[a].copy(),
                    tau=self.tau[a].copy(), tau_d=self.taud[a].copy(), ids=self.ids[a].copy(),
                    E=tuple(x.copy() for x in self.E), B=tuple(x.copy() for x in self.B),
                    j=tuple(x.copy() for x in self.j),
                    Te=self.Te.copy(), Ti=self.Ti.copy(), eta=self.eta.copy(),
                    ion_heat=self.ion_heat.copy(), step=self.step_index,
                    next_id=self.next_id, delta_next=self.delta_next)

    def set_state(self, st):
        self.X = np.array(st["pos"], dtype=np.float64).reshape(-1, 3) / self.dx
        self.p = np.array(st["p"], dtype=np.float64).reshape(-1, 3)
        self.w = np.array(st["w"], dtype=np.float64)
        self.tau = np.array(st["tau"], dtype=np.float64)
        self.ids = np.array(st["ids"], dtype=np.uint32)
        if st.get("tau_d") is not None:
            self.taud = np.array(st["tau_d"], dtype=np.float64)
        elif int(self.cfg["physics"]) & PHYS_DELTA:
            raise ValueError("delta rays need the electrons' tau_d")
        else:
            self.taud = np.zeros(len(self.ids))
        order = np.argsort(self.ids, kind="stable")
        self.X, self.p, self.w, self.tau, self.taud, self.ids = (
            a[order] for a in (self.X, self.p, self.w, self.tau, self.taud, self.ids))
        self.alive = np.ones(len(self.ids), dtype=bool)
        for key in ("E", "B"):
            if key in st and st[key] is not None:
                setattr(self, key, tuple(np.array(x, dtype=np.float64) for x in st[key]))
        for key in ("Te", "Ti", "eta"):
            if key in st and st[key] is not None:
                setattr(self, key, np.array(st[key], dtype=np.float64))
        if "step" in st:
            self.step_index = int(st["step"])
        if "next_id" in st:
            self.next_id = int(st["next_id"])
        if "delta_next" in st:
            self.delta_next = int(st["delta_next"])
