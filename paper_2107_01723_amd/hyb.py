"""Thin Python binding of the hybrid-PIC C ABI (include/hyb.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libhyb.so.  PyTorch provides the device memory (through the caching
allocator) and the stream.  If the library is not built the import of a run
fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyb.so")

HYB_OK, HYB_EINVAL, HYB_ENOMEM, HYB_ENOSPACE, HYB_EDEVICE, HYB_ESTATE, HYB_ENUMERIC, HYB_EBUSY = range(8)
FP64, FP32_MIXED = 0, 1
LEDGER_KEYS = ("injected", "field_loss", "field_gain", "ionisation", "stopped",
               "rad_discrete", "rad_subcut", "escaped", "reflux", "photon_thr", "residual")
COUNTER_KEYS = ("n_injected", "n_emitted", "n_reflux", "n_escaped", "n_stopped", "n_delta",
                "n_delta_lost", "n_electron_steps", "n_injection_lost")
PHYS_DELTA = 1 << 8
PHYS_URBAN = 1 << 9
DELTA_ID_BIT = 0x80000000

ABI_FUNCTIONS = (
    "hyb_init", "hyb_inject", "hyb_inject_envelope", "hyb_inject_beam", "hyb_step", "hyb_tally", "hyb_get_state", "hyb_set_state",
    "hyb_run_info_get", "hyb_table_get", "hyb_timing_enable", "hyb_timing_get", "hyb_use_graph",
    "hyb_footprint", "hyb_free", "hyb_last_error", "hyb_status_string", "hyb_abi_sizes", "hyb_model_scan",
    "hyb_model_scan_static",
    "hyb_engine_create", "hyb_engine_admit", "hyb_engine_step", "hyb_engine_poll",
    "hyb_engine_retire", "hyb_engine_stats", "hyb_engine_free",
)


class HybError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double),
        ("precision", C.c_int32),
        ("Z", C.c_double), ("A", C.c_double), ("rho", C.c_double),
        ("I_ex", C.c_double),
        ("x_lo", C.c_double), ("x_hi", C.c_double),
        ("T0", C.c_double),
        ("lambda1", C.c_double), ("lambda2", C.c_double),
        ("I0", C.c_double), ("wavelength", C.c_double),
        ("kappa_esc", C.c_double), ("kappa_tnsa", C.c_double), ("sigma_dtheta", C.c_double),
        ("reflux_ke_frac", C.c_double),
        ("brem_boost", C.c_double), ("k_cut", C.c_double),
        ("table_shape", C.c_int32), ("table_nT", C.c_int32), ("table_nr", C.c_int32),
        ("table_emax", C.c_double),
        ("e_min", C.c_double),
        ("tally_nE", C.c_int32), ("tally_ntheta", C.c_int32),
        ("tally_Elo", C.c_double), ("tally_Ehi", C.c_double),
        ("tally_Ethr", C.c_double),
        ("series_len", C.c_int32),
        ("seed", C.c_uint32),
        ("max_particles", C.c_int64),
        ("physics", C.c_uint32),
        ("eta_fixed", C.c_double),
        ("n_sub", C.c_int32),
        ("sort_every", C.c_int32),
        ("delta_cut", C.c_double),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("bc_z", C.c_int32),
        ("n_extra", C.c_int32), ("extra_Z", C.c_double * 3), ("extra_A", C.c_double * 3),
        ("extra_rho", C.c_double * 3), ("extra_I_ex", C.c_double * 3),
    ]


class Source(C.Structure):
    _fields_ = [
        ("n_macro", C.c_int64),
        ("t_start", C.c_double), ("t_end", C.c_double),
        ("y0", C.c_double), ("z0", C.c_double),
        ("r_fwhm", C.c_double), ("T_hot", C.c_double), ("half_angle", C.c_double),
        ("eta_l2e", C.c_double), ("weight", C.c_double),
    ]


class Envelope(C.Structure):
    _fields_ = [
        ("per_cell", C.c_int32),
        ("t_peak", C.c_double), ("t_fwhm", C.c_double),
        ("y0", C.c_double), ("z0", C.c_double), ("r_fwhm", C.c_double),
        ("g_min", C.c_double), ("f_min", C.c_double),
        ("max_half_angle", C.c_double), ("eta_l2e", C.c_double),
    ]


class Beam(C.Structure):
    _fields_ = [("per_cell", C.c_int32), ("t_start", C.c_double), ("energy", C.c_double),
                ("weight", C.c_double)]


class Model(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("wavelength", "eta_l2e", "r_fwhm", "t_fwhm", "fg_mean",
                                           "sqrt_fg_mean", "kappa_esc", "kappa_tnsa", "e_th", "Lx", "Ly",
                                           "Lz", "theta_c", "eta_mean", "n_i")] + [("nsteps", C.c_int32)]


MODEL_KEYS = ("brem", "photon_thr", "ionisation", "reflux", "field", "escaped")


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Device(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("user", C.c_void_p)]


class TallyOut(C.Structure):
    _fields_ = [
        ("hist_E", C.POINTER(C.c_double)), ("hist_N", C.POINTER(C.c_double)),
        ("series", C.POINTER(C.c_double)),
        ("flow", C.c_double * 4), ("ledger", C.c_double * 11),
        ("kinetic", C.c_double), ("conversion", C.c_double),
        ("counters", C.c_int64 * 9), ("n_alive", C.c_int64), ("step", C.c_int64),
    ]


class State(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("capacity", C.c_int64),
        ("pos", C.POINTER(C.c_double)), ("mom", C.POINTER(C.c_double)),
        ("w", C.POINTER(C.c_double)), ("tau", C.POINTER(C.c_double)),
        ("id", C.POINTER(C.c_uint32)),
        ("E", C.POINTER(C.c_double)), ("B", C.POINTER(C.c_double)), ("J", C.POINTER(C.c_double)),
        ("Te", C.POINTER(C.c_double)), ("Ti", C.POINTER(C.c_double)), ("eta", C.POINTER(C.c_double)),
        ("ion_heat", C.POINTER(C.c_double)),
        ("step", C.c_int64), ("next_id", C.c_int64),
        ("tau_d", C.POINTER(C.c_double)), ("delta_next", C.c_int64),
    ]


class RunInfo(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("a0", C.c_double), ("eps_esc", C.c_double),
                ("n_i", C.c_double), ("c_z", C.c_double), ("w_ref", C.c_double),
                ("nodes", C.c_int64), ("cells", C.c_int64), ("bytes", C.c_int64)]


_lib = None


def lib():
    """Load libhyb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2107_01723_amd.build`")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes libhyb.so bind to that one runtime, so torch's streams and
    # allocations are valid in the library.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sig = {
        "hyb_init": (C.c_int, [P(Config), P(Device), P(vp)]),
        "hyb_inject": (C.c_int, [vp, P(Source)]),
        "hyb_inject_envelope": (C.c_int, [vp, P(Envelope)]),
        "hyb_inject_beam": (C.c_int, [vp, P(Beam)]),
        "hyb_model_scan": (C.c_int, [P(Model), P(C.c_double), P(C.c_double), C.c_int64, P(C.c_double), vp]),
        "hyb_model_scan_static": (C.c_int, [P(Model), P(C.c_double), P(C.c_double), C.c_int64, P(C.c_double),
                                            vp]),
        "hyb_step": (C.c_int, [vp, C.c_int32]),
        "hyb_tally": (C.c_int, [vp, P(TallyOut)]),
        "hyb_get_state": (C.c_int, [vp, P(State)]),
        "hyb_set_state": (C.c_int, [vp, P(State)]),
        "hyb_run_info_get": (C.c_int, [vp, P(RunInfo)]),
        "hyb_table_get": (C.c_int, [vp, P(C.c_double), P(C.c_double), P(C.c_double)]),
        "hyb_timing_enable": (C.c_int, [vp, C.c_int32]),
        "hyb_timing_get": (C.c_int, [vp, P(C.c_double), P(C.c_int64)]),
        "hyb_use_graph": (C.c_int, [vp, C.c_int32]),
        "hyb_footprint": (C.c_int, [P(Config), P(C.c_int64)]),
        "hyb_free": (None, [vp]),
        "hyb_last_error": (C.c_char_p, [vp]),
        "hyb_status_string": (C.c_char_p, [C.c_int]),
        "hyb_abi_sizes": (None, [P(C.c_int64)]),
        "hyb_engine_create": (C.c_int, [P(Device), C.c_int64, C.c_int32, P(vp)]),
        "hyb_engine_admit": (C.c_int, [vp, P(Config), P(Source), C.c_int32, C.c_int32, P(vp)]),
        "hyb_engine_step": (C.c_int, [vp, C.c_int32]),
        "hyb_engine_poll": (C.c_int, [vp, P(vp), C.c_int32, P(C.c_int32)]),
        "hyb_engine_retire": (C.c_int, [vp, vp]),
        "hyb_engine_stats": (C.c_int, [vp, P(C.c_int32), P(C.c_int64), P(C.c_int64)]),
        "hyb_engine_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check_abi():
    """Compare the ctypes struct sizes with the library's."""
    a = (C.c_int64 * 9)()
    lib().hyb_abi_sizes(a)
    mine = [C.sizeof(t) for t in (Config, Source, Device, TallyOut, State, RunInfo, Envelope, Beam, Model)]
    if list(a) != mine:
        raise RuntimeError(f"ABI struct sizes differ: library {list(a)} binding {mine}")
    return mine


# config keys a dictionary may leave out, with their defaults
CONFIG_DEFAULTS = {"delta_cut": 1e3 * 1.602176634e-19, "bc_x": 0, "bc_y": 0, "bc_z": 0, "n_extra": 0,
                   "extra_Z": (0.0, 0.0, 0.0), "extra_A": (0.0, 0.0, 0.0), "extra_rho": (0.0, 0.0, 0.0),
                   "extra_I_ex": (0.0, 0.0, 0.0)}


def make_config(d: dict) -> Config:
    c = Config()
    for name, typ in Config._fields_:
        v = d[name] if name in d else CONFIG_DEFAULTS[name]
        if issubclass(typ, C.Array):
            v = typ(*[float(x) for x in v])
        setattr(c, name, v)
    return c


def make_source(d: dict) -> Source:
    s = Source()
    for name, _ in Source._fields_:
        setattr(s, name, d[name])
    return s


def make_envelope(d: dict) -> Envelope:
    e = Envelope()
    for name, _ in Envelope._fields_:
        setattr(e, name, d[name])
    return e


def footprint(cfg: dict) -> int:
    b = C.c_int64(0)
    st = lib().hyb_footprint(C.byref(make_config(cfg)), C.byref(b))
    if st != HYB_OK:
        raise HybError(st, lib().hyb_last_error(None).decode())
    return int(b.value)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def model_scan(m: dict, I0, Z, device: int = 0, stream=None):
    """The energy-partition model of Sec. III.B at the scan points (I0
    [W/m^2], Z) through hyb_model_scan.  Returns an array [6, n] of energy
    fractions in the order of MODEL_KEYS."""
    I0 = np.ascontiguousarray(np.asarray(I0, dtype=np.float64).ravel())
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).ravel())
    if I0.shape != Z.shape:
        raise ValueError("I0 and Z differ in length")
    mod = Model()
    for name, _ in Model._fields_:
        setattr(mod, name, m[name])
    out = np.zeros(6 * len(I0))
    dev, mem, _ = _device(device, stream, True)
    st = lib().hyb_model_scan(C.byref(mod), _dptr(I0), _dptr(Z), len(I0), _dptr(out), C.byref(dev))
    del mem
    if st != HYB_OK:
        raise HybError(st, "hyb_model_scan: " + lib().hyb_last_error(None).decode())
    return out.reshape(len(I0), 6).T.copy()


def model_scan_static(m: dict, I0, Z, device: int = 0, stream=None):
    """The same scan through hyb_model_scan_static, which stages through the
    library's per-GPU device array and allocates no device memory (at most
    65536 points).  Returns an array [6, n] like model_scan."""
    I0 = np.ascontiguousarray(np.asarray(I0, dtype=np.float64).ravel())
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).ravel())
    if I0.shape != Z.shape:
        raise ValueError("I0 and Z differ in length")
    mod = Model()
    for name, _ in Model._fields_:
        setattr(mod, name, m[name])
    out = np.zeros(6 * len(I0))
    dev = Device()
    dev.device = device
    dev.stream = stream
    st = lib().hyb_model_scan_static(C.byref(mod), _dptr(I0), _dptr(Z), len(I0), _dptr(out), C.byref(dev))
    if st != HYB_OK:
        raise HybError(st, "hyb_model_scan_static: " + lib().hyb_last_error(None).decode())
    return out.reshape(len(I0), 6).T.copy()


class _TorchMemory:
    """Device allocator callbacks routed to torch's caching allocator."""

    def __init__(self, device: int, stream):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            return int(self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
        except Exception:
            return None

    def _free(self, ptr, user):
        # a run still open at interpreter exit is freed after torch has
        # begun tearing down; the process releases that memory anyway
        cuda = getattr(self._torch, "cuda", None)
        if cuda is None or sys.is_finalizing():
            return
        cuda.caching_allocator_delete(ptr)


def _device(device: int, stream=None, torch_alloc=True):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    mem = _TorchMemory(device, stream) if torch_alloc else None
    dev = Device()
    dev.device = device
    dev.stream = C.c_void_p(stream.cuda_stream)
    if mem is not None:
        dev.alloc = mem.alloc
        dev.free = mem.free
    dev.user = None
    return dev, mem, stream


class Run:
    """One hybrid-PIC run on the GPU (hyb_init ... hyb_free)."""

    def __init__(self, cfg: dict, device: int = 0, stream=None, torch_alloc: bool = True):
        self.L = lib()
        self.cfg = dict(cfg)
        self._dev, self._mem, self.stream = _device(device, stream, torch_alloc)
        h = C.c_void_p()
        st = self.L.hyb_init(C.byref(make_config(cfg)), C.byref(self._dev), C.byref(h))
        if st != HYB_OK:
            raise HybError(st, "hyb_init: " + self.L.hyb_last_error(None).decode())
        self.h = h
        self._engine = None

    @classmethod
    def _from_engine(cls, engine, handle, cfg):
        self = cls.__new__(cls)
        self.L = lib()
        self.cfg = dict(cfg)
        self._dev, self._mem, self.stream = engine._dev, engine._mem, engine.stream
        self.h = handle
        self._engine = engine
        return self

    def _check(self, st, what):
        if st != HYB_OK:
            raise HybError(st, f"{what}: " + self.L.hyb_last_error(self.h).decode())

    def inject(self, src: dict):
        self._check(self.L.hyb_inject(self.h, C.byref(make_source(src))), "hyb_inject")

    def inject_envelope(self, env: dict):
        """The paper's envelope injection (hyb_inject_envelope)."""
        self._check(self.L.hyb_inject_envelope(self.h, C.byref(make_envelope(env))), "hyb_inject_envelope")

    def inject_beam(self, beam: dict):
        """A mono-energetic normal-incidence beam (hyb_inject_beam)."""
        b = Beam()
        for name, _ in Beam._fields_:
            setattr(b, name, beam[name])
        self._check(self.L.hyb_inject_beam(self.h, C.byref(b)), "hyb_inject_beam")

    def step(self, n: int = 1):
        self._check(self.L.hyb_step(self.h, int(n)), "hyb_step")

    def use_graph(self, on: bool = True):
        self._check(self.L.hyb_use_graph(self.h, 1 if on else 0), "hyb_use_graph")

    def timing(self, on: bool = True):
        self._check(self.L.hyb_timing_enable(self.h, 1 if on else 0), "hyb_timing_enable")

    def timing_get(self):
        ms = C.c_double(0)
        n = C.c_int64(0)
        self._check(self.L.hyb_timing_get(self.h, C.byref(ms), C.byref(n)), "hyb_timing_get")
        return float(ms.value), int(n.value)

    def info(self) -> dict:
        i = RunInfo()
        self._check(self.L.hyb_run_info_get(self.h, C.byref(i)), "hyb_run_info_get")
        return {name: getattr(i, name) for name, _ in RunInfo._fields_}

    def table(self):
        nT, nr = int(self.cfg["table_nT"]), int(self.cfg["table_nr"])
        X = np.zeros(nT * nr)
        S = np.zeros(nT)
        U = np.zeros(nT)
        self._check(self.L.hyb_table_get(self.h, _dptr(X), _dptr(S), _dptr(U)), "hyb_table_get")
        return X.reshape(nT, nr), S, U

    def tally(self) -> dict:
        c = self.cfg
        nE, nth = int(c["tally_nE"]), int(c["tally_ntheta"])
        hE = np.zeros(nE * nth)
        hN = np.zeros(nE * nth)
        ser = np.zeros(max(1, int(c["series_len"])))
        out = TallyOut()
        out.hist_E = _dptr(hE)
        out.hist_N = _dptr(hN)
        out.series = _dptr(ser)
        self._check(self.L.hyb_tally(self.h, C.byref(out)), "hyb_tally")
        return dict(hist_E=hE.reshape(nE, nth), hist_N=hN.reshape(nE, nth),
                    series=ser[: int(c["series_len"])], flow=np.array(out.flow[:]),
                    ledger={k: out.ledger[i] for i, k in enumerate(LEDGER_KEYS)},
                    counters={k: int(out.counters[i]) for i, k in enumerate(COUNTER_KEYS)},
                    kinetic=out.kinetic, conversion=out.conversion, n_alive=int(out.n_alive),
                    step=int(out.step))

    def get_state(self, capacity: int | None = None) -> dict:
        c = self.cfg
        nodes = (c["nx"] + 1) * (c["ny"] + 1) * (c["nz"] + 1)
        cells = c["nx"] * c["ny"] * c["nz"]
        cap = int(capacity if capacity is not None else c["max_particles"])
        a = dict(pos=np.zeros(3 * cap), mom=np.zeros(3 * cap), w=np.zeros(cap), tau=np.zeros(cap),
                 tau_d=np.zeros(cap), id=np.zeros(cap, dtype=np.uint32), E=np.zeros(3 * nodes), B=np.zeros(3 * nodes),
                 J=np.zeros(3 * nodes), Te=np.zeros(cells), Ti=np.zeros(cells), eta=np.zeros(cells),
                 ion_heat=np.zeros(cells))
        s = State()
        s.capacity = cap
        for k in ("pos", "mom", "w", "tau", "tau_d", "E", "B", "J", "Te", "Ti", "eta", "ion_heat"):
            setattr(s, k, _dptr(a[k]))
        s.id = a["id"].ctypes.data_as(C.POINTER(C.c_uint32))
        self._check(self.L.hyb_get_state(self.h, C.byref(s)), "hyb_get_state")
        n = int(s.n)
        shp = (c["nz"] + 1, c["ny"] + 1, c["nx"] + 1)
        cshp = (c["nz"], c["ny"], c["nx"])

        def fld(v):   # -> tuple of 3 arrays indexed [i, j, k]
            return tuple(v[d * nodes:(d + 1) * nodes].reshape(shp).transpose(2, 1, 0).copy() for d in range(3))

        def cel(v):
            return v.reshape(cshp).transpose(2, 1, 0).copy()

        return dict(pos=a["pos"][: 3 * n].reshape(n, 3), p=a["mom"][: 3 * n].reshape(n, 3),
                    w=a["w"][:n], tau=a["tau"][:n], tau_d=a["tau_d"][:n], ids=a["id"][:n],
                    E=fld(a["E"]), B=fld(a["B"]), j=fld(a["J"]), Te=cel(a["Te"]), Ti=cel(a["Ti"]),
                    eta=cel(a["eta"]), ion_heat=cel(a["ion_heat"]), step=int(s.step),
                    next_id=int(s.next_id), delta_next=int(s.delta_next))

    def set_state(self, st: dict):
        """st: pos (n,3) m, p (n,3) kg m/s, w, tau, ids; tau_d with delta rays;
        optional E, B (3 arrays [i,j,k]), Te, Ti, eta ([i,j,k]); step, next_id,
        delta_next."""
        n = len(st["ids"])
        keep = []

        def arr(x, dt=np.float64):
            v = np.ascontiguousarray(np.asarray(x, dtype=dt).ravel())
            keep.append(v)
            return v

        s = State()
        s.n = n
        s.capacity = n
        pos, mom = arr(st["pos"]), arr(st["p"])
        w, tau = arr(st["w"]), arr(st["tau"])
        ids = arr(st["ids"], np.uint32)
        s.pos, s.mom, s.w, s.tau = _dptr(pos), _dptr(mom), _dptr(w), _dptr(tau)
        s.id = ids.ctypes.data_as(C.POINTER(C.c_uint32))
        s.tau_d = _dptr(arr(st["tau_d"])) if st.get("tau_d") is not None else None

        def fld(t):
            return arr(np.concatenate([np.asarray(x).transpose(2, 1, 0).ravel() for x in t]))

        def cel(x):
            return arr(np.asarray(x).transpose(2, 1, 0).ravel())

        for k in ("E", "B"):
            setattr(s, k, _dptr(fld(st[k])) if st.get(k) is not None else None)
        for k in ("Te", "Ti", "eta"):
            setattr(s, k, _dptr(cel(st[k])) if st.get(k) is not None else None)
        s.J = None
        s.ion_heat = None
        s.step = int(st.get("step", 0))
        s.next_id = int(st.get("next_id", 0))
        s.delta_next = int(st.get("delta_next", 0))
        self._check(self.L.hyb_set_state(self.h, C.byref(s)), "hyb_set_state")

    def close(self):
        if getattr(self, "h", None) and self._engine is None:
            self.L.hyb_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Continuous-batching engine (hyb_engine_*)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, max_runs: int = 64, stream=None,
                 torch_alloc: bool = True):
        self.L = lib()
        self._dev, self._mem, self.stream = _device(device, stream, torch_alloc)
        h = C.c_void_p()
        st = self.L.hyb_engine_create(C.byref(self._dev), int(hbm_budget), int(max_runs), C.byref(h))
        if st != HYB_OK:
            raise HybError(st, "hyb_engine_create: " + self.L.hyb_last_error(None).decode())
        self.h = h
        self.max_runs = max_runs
        self.runs = {}

    def admit(self, cfg: dict, srcs: list, nsteps: int):
        """Returns a Run handle, or None when the engine is busy (no slot or memory)."""
        arr = (Source * max(1, len(srcs)))(*[make_source(s) for s in srcs])
        h = C.c_void_p()
        st = self.L.hyb_engine_admit(self.h, C.byref(make_config(cfg)), arr, len(srcs), int(nsteps),
                                     C.byref(h))
        if st == HYB_EBUSY:
            return None
        if st != HYB_OK:
            raise HybError(st, "hyb_engine_admit: " + self.L.hyb_last_error(None).decode())
        r = Run._from_engine(self, h, cfg)
        self.runs[h.value] = r
        return r

    def step(self, nticks: int = 1):
        st = self.L.hyb_engine_step(self.h, int(nticks))
        if st != HYB_OK:
            raise HybError(st, "hyb_engine_step: " + self.L.hyb_last_error(None).decode())

    def poll(self):
        buf = (C.c_void_p * self.max_runs)()
        n = C.c_int32(0)
        st = self.L.hyb_engine_poll(self.h, buf, self.max_runs, C.byref(n))
        if st != HYB_OK:
            raise HybError(st, "hyb_engine_poll: " + self.L.hyb_last_error(None).decode())
        return [self.runs[buf[i]] for i in range(n.value)]

    def retire(self, run: Run):
        st = self.L.hyb_engine_retire(self.h, run.h)
        if st != HYB_OK:
            raise HybError(st, "hyb_engine_retire: " + self.L.hyb_last_error(None).decode())
        self.runs.pop(run.h.value, None)
        run.h = None

    def stats(self):
        n = C.c_int32(0)
        u = C.c_int64(0)
        b = C.c_int64(0)
        self.L.hyb_engine_stats(self.h, C.byref(n), C.byref(u), C.byref(b))
        return dict(resident=n.value, bytes_used=u.value, budget=b.value)

    def close(self):
        if getattr(self, "h", None):
            self.L.hyb_engine_free(self.h)
            self.h = None
            for r in self.runs.values():
                r.h = None
            self.runs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
