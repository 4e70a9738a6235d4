"""FP64 CPU oracle for the 1D3V electrostatic PIC-MCC step (ctypes binding).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The GPU library never imports it.

The arithmetic lives in ``pic_oracle.c`` (plain C, FP64, -ffp-contract=off);
this module only marshals numpy arrays.  Every function there cites the part
of the paper (arXiv 2404.10270, Sec. 2 phase list and the moveb listing of
Sec. 6) or the published method it follows.

Parity unpinned (no closed form or published value exists; only the
invariants listed in the tests constrain them): the warm-plasma Langmuir
dispersion beyond the cold limit, and the long-time sheath evolution of the
bounded workloads.  The cross-section values are configuration inputs, not
physics claims.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time
from typing import List, Optional

import numpy as np

import pic_inputs as pin

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "libpic_oracle.so")

MAXSP = 4
XS_IZ_RATE = 1          # ionisation with a constant rate coefficient sig_iz v_cap
ST_CAPACITY, ST_CFL, ST_NN_CAP = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction of multiply-adds)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


class Config(C.Structure):
    _fields_ = [("nc", C.c_int32), ("bc", C.c_int32), ("nsp", C.c_int32), ("mcc_on", C.c_int32),
                ("source_on", C.c_int32), ("inst", C.c_int32), ("seed", C.c_uint64),
                ("dx", C.c_double), ("dt", C.c_double), ("eps0", C.c_double),
                ("B0", C.c_double), ("theta", C.c_double),
                ("q", C.c_double * MAXSP), ("m", C.c_double * MAXSP), ("w", C.c_double * MAXSP),
                ("kind", C.c_int32 * MAXSP), ("nstep", C.c_int32 * MAXSP),
                ("v_cap", C.c_double * MAXSP), ("T_src", C.c_double * MAXSP),
                ("n_n", C.c_double), ("T_n", C.c_double), ("sig_el", C.c_double),
                ("sig_iz", C.c_double), ("E_iz", C.c_double), ("sig_cx", C.c_double),
                ("smooth_passes", C.c_int32), ("_pad", C.c_int32),
                ("sig_ex", C.c_double), ("E_ex", C.c_double), ("field_off", C.c_int32),
                ("xs_flags", C.c_uint32)]


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64),
                ("x", C.POINTER(C.c_double)), ("vx", C.POINTER(C.c_double)),
                ("vy", C.POINTER(C.c_double)), ("vz", C.POINTER(C.c_double)),
                ("id", C.POINTER(C.c_uint64))]


class Counters(C.Structure):
    _fields_ = [("step", C.c_int64), ("next_id", C.c_uint64), ("status", C.c_uint32),
                ("_pad", C.c_uint32),
                ("absorbed", (C.c_int64 * 2) * MAXSP),
                ("absorbed_total", (C.c_int64 * 2) * MAXSP),
                ("created_total", C.c_int64 * MAXSP),
                ("n_candidates", C.c_int64), ("n_elastic", C.c_int64), ("n_ionize", C.c_int64),
                ("n_cx", C.c_int64), ("n_over_cap", C.c_int64), ("n_source", C.c_int64),
                ("particle_steps", C.c_int64),
                ("n_excite", C.c_int64), ("n_consumed", C.c_int64),
                ("n_iz_untargeted", C.c_int64)]


class Sim(C.Structure):
    _fields_ = [("cfg", Config), ("sp", Particles * MAXSP), ("cnt", Counters),
                ("S", C.POINTER(C.c_uint64) * MAXSP),
                ("rho", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
                ("E", C.POINTER(C.c_double)),
                ("acc", C.POINTER(C.c_double) * MAXSP),
                ("nn", C.POINTER(C.c_double))]


class Diag(C.Structure):
    _fields_ = [("n", C.c_int64 * MAXSP), ("ke", C.c_double * MAXSP),
                ("mom", (C.c_double * 3) * MAXSP), ("field_energy", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint64)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_deposit_species.argtypes = [C.c_int64, dp, C.c_int32, up]
        L.orc_deposit_cic64.argtypes = [C.c_int64, dp, C.c_int32, dp]
        L.orc_thomas.argtypes = [C.c_int64, dp, dp, dp, dp, dp]
        L.orc_thomas.restype = C.c_int
        L.orc_poisson_dirichlet.argtypes = [C.c_int64, dp, dp]
        L.orc_smooth.argtypes = [C.c_int32, C.c_int, C.c_int, dp, dp]
        L.orc_smooth.restype = None
        L.orc_poisson_dirichlet.restype = C.c_int
        for name in ("orc_deposit", "orc_push", "orc_walls"):
            getattr(L, name).argtypes = [C.POINTER(Sim)]
            getattr(L, name).restype = None
        for name in ("orc_field", "orc_mcc", "orc_source", "orc_step"):
            getattr(L, name).argtypes = [C.POINTER(Sim)]
            getattr(L, name).restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(Sim), C.c_int64]
        L.orc_run.restype = C.c_int
        L.orc_diagnostics.argtypes = [C.POINTER(Sim), C.POINTER(Diag)]
        ip = C.POINTER(C.c_int64)
        L.orc_init_species.argtypes = [C.POINTER(Config), ip, C.c_int, C.c_int, C.c_int,
                                       C.c_double, C.c_int, dp, C.c_int64, ip, dp, dp, dp, dp, up]
        L.orc_init_species.restype = None
        L.orc_init_deposit.argtypes = [C.POINTER(Config), ip, C.c_int, C.c_int, C.c_int,
                                       C.c_double, C.c_int, C.c_int, up]
        L.orc_init_deposit.restype = None
        L.orc_fp32_form.argtypes = [C.c_double, C.c_int32]
        L.orc_fp32_form.restype = C.c_double
        L.orc_candidate_threshold.argtypes = [C.POINTER(Config), C.c_int]
        L.orc_candidate_threshold.restype = C.c_uint64
        L.orc_neutral_key.argtypes = [C.POINTER(Config), C.c_uint64, C.c_int64]
        L.orc_neutral_key.restype = C.c_uint64
        for name, T in (("orc_sizeof_sim", Sim), ("orc_sizeof_config", Config),
                        ("orc_sizeof_counters", Counters), ("orc_sizeof_diag", Diag)):
            f = getattr(L, name)
            f.restype = C.c_int
            if f() != C.sizeof(T):
                raise RuntimeError(f"oracle struct layout mismatch for {T.__name__}")
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = C.c_int
        L.orc_set_threads(1)  # one thread unless set_threads asks for more
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads for the oracle's independent per-particle loops (results are
    bit-identical for any count); returns the count in effect."""
    lib().orc_set_threads(int(n))
    return int(lib().orc_get_threads())


def threads() -> int:
    return int(lib().orc_get_threads())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


# ---------------------------------------------------------------------------
# small entry points used by the pins
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def deposit_fixed(x: np.ndarray, nc: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    S = np.zeros(nc + 1, dtype=np.uint64)
    lib().orc_deposit_species(x.shape[0], _dp(x), nc, _up(S))
    return S


def deposit_cic64(x: np.ndarray, nc: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(nc + 1, dtype=np.float64)
    lib().orc_deposit_cic64(x.shape[0], _dp(x), nc, _dp(out))
    return out


def thomas(a, b, c, d) -> np.ndarray:
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    x = np.zeros_like(d)
    rc = lib().orc_thomas(d.shape[0], _dp(a), _dp(b), _dp(c), _dp(d), _dp(x))
    if rc:
        raise MemoryError("orc_thomas")
    return x


def smooth(rho, V, bc: int, passes: int) -> np.ndarray:
    """The density smoother applied to a copy of rho (nodes 0..nc, volumes V)."""
    r = np.array(rho, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    lib().orc_smooth(r.shape[0] - 1, int(bc), int(passes), _dp(V), _dp(r))
    return r


def fp32_form(x: float, nc: int) -> float:
    """The value of position x (cells) as stored in the FP32 form (orc_fp32_form)."""
    return float(lib().orc_fp32_form(float(x), int(nc)))


def poisson_dirichlet(d) -> np.ndarray:
    """Solve tridiag(1, -2, 1) x = d (Dirichlet ends) with the closed-form pivots."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    x = np.zeros_like(d)
    if lib().orc_poisson_dirichlet(d.shape[0], _dp(d), _dp(x)):
        raise MemoryError("orc_poisson_dirichlet")
    return x


# ---------------------------------------------------------------------------
# the simulation object
# ---------------------------------------------------------------------------

def make_config(wl: pin.Workload, inst: int = 0) -> Config:
    c = Config()
    c.nc = wl.nc
    c.bc = wl.bc
    c.nsp = len(wl.species)
    c.mcc_on = 1 if wl.mcc is not None else 0
    c.source_on = 1 if wl.source else 0
    c.inst = inst
    c.seed = wl.seed
    c.dx, c.dt, c.eps0, c.B0, c.theta = wl.dx, wl.dt, wl.eps0, wl.B0, wl.theta
    for k, s in enumerate(wl.species):
        c.q[k], c.m[k], c.w[k] = s.q, s.m, s.w
        c.kind[k] = s.kind
        c.nstep[k] = int(getattr(s, "nstep", 1))
        c.v_cap[k] = s.v_cap
        c.T_src[k] = s.T_src
    c.smooth_passes = int(getattr(wl, "smooth_passes", 0))
    c.field_off = 1 if wl.field_off else 0
    if wl.mcc is not None:
        mc = wl.mcc
        c.n_n, c.T_n, c.sig_el, c.sig_iz, c.E_iz, c.sig_cx = (mc.n_n, mc.T_n, mc.sig_el,
                                                               mc.sig_iz, mc.E_iz, mc.sig_cx)
        c.sig_ex, c.E_ex = mc.sig_ex, mc.E_ex
        c.xs_flags = XS_IZ_RATE if mc.iz_const_rate else 0
    return c


def _init_args(wl: pin.Workload, inst: int):
    c = make_config(wl, inst)
    nsp = len(wl.species)
    n_init = (C.c_int64 * MAXSP)(*([int(round(s.ppc * wl.nc)) for s in wl.species]
                                   + [0] * (MAXSP - nsp)))
    T = np.zeros(MAXSP)
    for k, s in enumerate(wl.species):
        T[k] = s.T
    opts = (1 if wl.quiet else 0, 1 if wl.pair_start else 0, float(wl.perturb_amp),
            int(wl.perturb_mode))
    return c, n_init, T, opts


def init_state(wl: pin.Workload, inst: int = 0, select=None) -> List[pin.SpeciesState]:
    """The configuration's own initial particles, drawn from the counter-based
    generator at step -1 (orc_init_species): round(ppc nc) particles per
    species, ids counting from 0 over the species in order.  `select`, if
    given, lists per species the particle indices to draw (a sample)."""
    c, n_init, T, opts = _init_args(wl, inst)
    out = []
    for k in range(len(wl.species)):
        if select is None:
            m, plist, pp = n_init[k], None, None
        else:
            pp = np.ascontiguousarray(select[k], dtype=np.int64)
            m, plist = pp.shape[0], pp.ctypes.data_as(C.POINTER(C.c_int64))
        x = np.zeros(m); vx = np.zeros(m); vy = np.zeros(m); vz = np.zeros(m)
        ids = np.zeros(m, dtype=np.uint64)
        lib().orc_init_species(C.byref(c), n_init, k, *opts, _dp(T), m, plist, _dp(x), _dp(vx),
                               _dp(vy), _dp(vz), _up(ids))
        out.append(pin.SpeciesState(x=x, vx=vx, vy=vy, vz=vz, id=ids))
    return out


def init_deposit(wl: pin.Workload, inst: int = 0, fp32_form: bool = False) -> List[np.ndarray]:
    """Fixed-point deposit of every drawn initial particle, per species,
    computed particle by particle (no particle arrays are stored); with
    fp32_form the positions are first rounded to the FP32 storage form."""
    c, n_init, T, opts = _init_args(wl, inst)
    out = []
    for k in range(len(wl.species)):
        S = np.zeros(wl.nc + 1, dtype=np.uint64)
        lib().orc_init_deposit(C.byref(c), n_init, k, *opts, 1 if fp32_form else 0, _up(S))
        out.append(S)
    return out


class OracleSim:
    """Owns numpy buffers and a ``Sim`` struct pointing into them."""

    def __init__(self, wl: pin.Workload, state: List[pin.SpeciesState],
                 caps: Optional[List[int]] = None, inst: int = 0):
        self.wl = wl
        nsp = len(wl.species)
        if nsp > MAXSP:
            raise ValueError("too many species")
        if caps is None:
            caps = pin.capacities(wl, state)
        self.sim = Sim()
        self.sim.cfg = make_config(wl, inst)
        self.arrays = []
        nc = wl.nc
        self.x, self.vx, self.vy, self.vz, self.id = [], [], [], [], []
        for k in range(nsp):
            st = state[k]
            cap = max(int(caps[k]), st.n, 1)
            x = np.zeros(cap); vx = np.zeros(cap); vy = np.zeros(cap); vz = np.zeros(cap)
            ids = np.zeros(cap, dtype=np.uint64)
            x[:st.n] = st.x; vx[:st.n] = st.vx; vy[:st.n] = st.vy; vz[:st.n] = st.vz
            ids[:st.n] = st.id
            P = self.sim.sp[k]
            P.n, P.cap = st.n, cap
            P.x, P.vx, P.vy, P.vz, P.id = _dp(x), _dp(vx), _dp(vy), _dp(vz), _up(ids)
            self.x.append(x); self.vx.append(vx); self.vy.append(vy); self.vz.append(vz)
            self.id.append(ids)
        self.S = [np.zeros(nc + 1, dtype=np.uint64) for _ in range(nsp)]
        self.acc = [np.zeros(nc + 1) for _ in range(nsp)]
        self.rho = np.zeros(nc + 1)
        self.phi = np.zeros(nc + 1)
        self.E = np.zeros(nc + 1)
        self.nn = np.zeros(nc + 1)
        self.sim.nn = _dp(self.nn)
        for k in range(nsp):
            self.sim.S[k] = _up(self.S[k])
            self.sim.acc[k] = _dp(self.acc[k])
        self.sim.rho, self.sim.phi, self.sim.E = _dp(self.rho), _dp(self.phi), _dp(self.E)
        self.sim.cnt.next_id = int(sum(st.n for st in state))
        self.sim.cnt.step = 0

    # -- phases ------------------------------------------------------------
    def deposit(self):
        lib().orc_deposit(C.byref(self.sim))

    def field(self):
        if lib().orc_field(C.byref(self.sim)):
            raise MemoryError("orc_field")

    def push(self):
        lib().orc_push(C.byref(self.sim))

    def walls(self):
        lib().orc_walls(C.byref(self.sim))

    def mcc(self):
        if lib().orc_mcc(C.byref(self.sim)):
            raise RuntimeError("orc_mcc")

    def source(self):
        if lib().orc_source(C.byref(self.sim)):
            raise RuntimeError("orc_source")

    def step(self, n: int = 1):
        if lib().orc_run(C.byref(self.sim), int(n)):
            raise RuntimeError("orc_run")

    # -- state ---------------------------------------------------------------
    @property
    def step_index(self) -> int:
        return int(self.sim.cnt.step)

    @property
    def counters(self) -> Counters:
        return self.sim.cnt

    def n(self, k: int) -> int:
        return int(self.sim.sp[k].n)

    def state(self, k: int) -> pin.SpeciesState:
        n = self.n(k)
        return pin.SpeciesState(x=self.x[k][:n].copy(), vx=self.vx[k][:n].copy(),
                                vy=self.vy[k][:n].copy(), vz=self.vz[k][:n].copy(),
                                id=self.id[k][:n].copy())

    def diagnostics(self) -> Diag:
        d = Diag()
        lib().orc_diagnostics(C.byref(self.sim), C.byref(d))
        return d

    def candidate_threshold(self, k: int) -> int:
        return int(lib().orc_candidate_threshold(C.byref(self.sim.cfg), k))

    def neutral_key(self, pid: int, step: int) -> int:
        """Order key of a kinetic neutral for consumption by ionisation at `step`."""
        return int(lib().orc_neutral_key(C.byref(self.sim.cfg), int(pid), int(step)))

    def snapshot(self):
        """Copy of everything that defines the future of the run."""
        return {"state": [self.state(k) for k in range(len(self.wl.species))],
                "step": self.step_index, "next_id": int(self.sim.cnt.next_id)}

    @classmethod
    def from_snapshot(cls, wl, snap, caps=None, inst=0):
        o = cls(wl, snap["state"], caps=caps, inst=inst)
        o.sim.cnt.step = snap["step"]
        o.sim.cnt.next_id = snap["next_id"]
        return o


def time_steps(wl: pin.Workload, state, n_steps: int, caps=None, n_threads: int = 1):
    """Wall-clock the oracle as it stands for n_steps on n_threads threads.

    Returns (particle_steps, seconds)."""
    prev = threads()
    set_threads(n_threads)
    try:
        o = OracleSim(wl, state, caps=caps)
        ps0 = int(o.sim.cnt.particle_steps)
        t0 = time.perf_counter()
        o.step(n_steps)
        dt = time.perf_counter() - t0
    finally:
        set_threads(prev)
    return int(o.sim.cnt.particle_steps) - ps0, dt
