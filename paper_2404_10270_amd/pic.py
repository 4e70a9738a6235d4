"""ctypes binding of libpic (include/pic.h): argument marshalling only.

The module-level functions carry the C ABI's names and signatures.  Device
memory comes from PyTorch (ROCm) tensors, the stream from
``torch.cuda.current_stream()``; every step of the method runs in libpic's
HIP kernels.  There is no CPU fallback: without the built library or a GPU
the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_MAX_SPECIES = 4
PIC_FRAC_BITS = 32

PIC_OK, PIC_E_ARG, PIC_E_CONFIG, PIC_E_DEVICE = 0, -1, -2, -3
PIC_E_CAPACITY, PIC_E_CFL, PIC_E_NONFINITE, PIC_E_STATE = -4, -5, -6, -7
PIC_E_SCRATCH, PIC_E_BUSY = -8, -9
PIC_STATIC_WORK_MAX = 64 << 20

PIC_ST_CAPACITY, PIC_ST_CFL, PIC_ST_NONFINITE = 0x1, 0x2, 0x4
PIC_ST_CANDIDATES, PIC_ST_INTERNAL, PIC_ST_BAD_INIT = 0x8, 0x10, 0x20
PIC_ST_NN_CAP = 0x40
PIC_XS_IZ_RATE = 0x1

PIC_BC_PERIODIC, PIC_BC_ABSORB = 0, 1
PIC_KIND_ELECTRON, PIC_KIND_ION, PIC_KIND_NEUTRAL = 0, 1, 2
PIC_FP32, PIC_FP64 = 0, 1

PIC_R_DEPOSIT, PIC_R_RHO, PIC_R_PHI, PIC_R_EFIELD = 0, 1, 2, 3
PIC_R_ACC64, PIC_R_ACC32, PIC_R_CELL_OFFSETS, PIC_R_NODE_BASE = 4, 5, 6, 7
PIC_R_NEUTRAL_DENSITY = 8

PIC_INIT_NO_FIELD = 0x1
PIC_INIT_SORT = 0x2
PIC_INIT_DEVICE = 0x4
PIC_INIT_OPT_QUIET, PIC_INIT_OPT_PAIR = 0x1, 0x2
PIC_PUSH_NO_DEPOSIT = 0x1

# every entry point declared in include/pic.h
ABI_SYMBOLS = ("pic_query_sizes", "pic_init", "pic_push", "pic_deposit", "pic_field_solve",
               "pic_mcc_collide", "pic_sort", "pic_diagnostics", "pic_step", "pic_step_graph",
               "pic_autotune_sort", "pic_region", "pic_destroy", "pic_strerror",
               "pic_init_static", "pic_set_mover", "pic_autotune")


class pic_species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double), ("kind", C.c_int32),
                ("nstep", C.c_int32), ("capacity", C.c_int64), ("n_init", C.c_int64),
                ("v_cap", C.c_double), ("T_src", C.c_double), ("T_init", C.c_double)]


class pic_config(C.Structure):
    _fields_ = [("nc", C.c_int32), ("bc", C.c_int32), ("nsp", C.c_int32),
                ("precision", C.c_int32), ("mcc_on", C.c_int32), ("source_on", C.c_int32),
                ("_pad0", C.c_int32), ("_pad1", C.c_int32), ("seed", C.c_uint64),
                ("dx", C.c_double), ("dt", C.c_double), ("eps0", C.c_double),
                ("B0", C.c_double), ("theta", C.c_double),
                ("sp", pic_species * PIC_MAX_SPECIES),
                ("n_n", C.c_double), ("T_n", C.c_double), ("sig_el", C.c_double),
                ("sig_iz", C.c_double), ("E_iz", C.c_double), ("sig_cx", C.c_double),
                ("next_id", C.c_uint64), ("step0", C.c_int64),
                ("init_amp", C.c_double), ("init_mode", C.c_int32), ("init_opts", C.c_uint32),
                ("smooth_passes", C.c_int32), ("_pad2", C.c_int32),
                ("sig_ex", C.c_double), ("E_ex", C.c_double), ("field_off", C.c_int32),
                ("xs_flags", C.c_uint32)]


class pic_sizes(C.Structure):
    _fields_ = [("n_slots", C.c_int64), ("n_segments", C.c_int64), ("n_nodes", C.c_int64),
                ("work_bytes", C.c_uint64), ("x_elem_bytes", C.c_int64),
                ("v_elem_bytes", C.c_int64), ("mover_blocks", C.c_int64),
                ("mover_blocks_max", C.c_int64)]


class pic_buffers(C.Structure):
    _fields_ = [("x", C.c_void_p * 2), ("cell", C.c_void_p * 2), ("vx", C.c_void_p * 2),
                ("vy", C.c_void_p * 2), ("vz", C.c_void_p * 2), ("id_lo", C.c_void_p * 2),
                ("id_hi", C.c_void_p * 2), ("work", C.c_void_p)]


class pic_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("next_id", C.c_uint64), ("status", C.c_uint32),
                ("cur_set", C.c_int32),
                ("n_slots_used", C.c_int64 * PIC_MAX_SPECIES),
                ("n_live", C.c_int64 * PIC_MAX_SPECIES),
                ("ke", C.c_double * PIC_MAX_SPECIES),
                ("mom", (C.c_double * 3) * PIC_MAX_SPECIES),
                ("field_energy", C.c_double),
                ("absorbed_total", (C.c_int64 * 2) * PIC_MAX_SPECIES),
                ("created_total", C.c_int64 * PIC_MAX_SPECIES),
                ("n_candidates", C.c_int64), ("n_elastic", C.c_int64), ("n_ionize", C.c_int64),
                ("n_cx", C.c_int64), ("n_over_cap", C.c_int64), ("n_source", C.c_int64),
                ("particle_steps", C.c_int64), ("n_excite", C.c_int64),
                ("n_consumed", C.c_int64), ("n_iz_untargeted", C.c_int64)]


class PicError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {pic_strerror(code)} ({code})")


_lib = None


def lib():
    """Load libpic.so (built in-tree).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2404_10270_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pic_query_sizes.argtypes = [C.POINTER(pic_config), C.c_int, C.POINTER(pic_sizes),
                                      C.POINTER(C.c_int64)]
        L.pic_init.argtypes = [C.POINTER(pic_config), C.c_int, C.POINTER(pic_buffers), P, C.c_uint,
                               C.POINTER(P)]
        L.pic_init_static.argtypes = L.pic_init.argtypes
        for name in ("pic_push",):
            getattr(L, name).argtypes = [P, C.c_uint]
        for name in ("pic_deposit", "pic_field_solve", "pic_mcc_collide", "pic_sort",
                     "pic_destroy"):
            getattr(L, name).argtypes = [P]
        L.pic_step.argtypes = [P, C.c_int, C.c_int]
        L.pic_step_graph.argtypes = [P, C.c_int, C.c_int]
        L.pic_autotune_sort.argtypes = [P, C.POINTER(C.c_int), C.c_int, C.c_int,
                                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.pic_set_mover.argtypes = [P, C.c_int, C.c_int]
        ip = C.POINTER(C.c_int)
        L.pic_autotune.argtypes = [P, ip, ip, C.c_int, ip, C.c_int, C.c_int, ip, ip,
                                   C.POINTER(C.c_double)]
        L.pic_diagnostics.argtypes = [P, C.POINTER(pic_diag), C.c_int]
        L.pic_region.argtypes = [P, C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_int64)]
        L.pic_strerror.argtypes = [C.c_int]
        L.pic_strerror.restype = C.c_char_p
        for name in ABI_SYMBOLS:
            if name != "pic_strerror":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise PicError(rc, what)
    return rc


# ---------------------------------------------------------------------------
# the ABI, same names
# ---------------------------------------------------------------------------

def pic_strerror(code: int) -> str:
    return lib().pic_strerror(int(code)).decode()


def pic_query_sizes(cfgs: Sequence[pic_config]):
    arr = (pic_config * len(cfgs))(*cfgs)
    out = pic_sizes()
    nsp = cfgs[0].nsp if len(cfgs) else 0
    seg = (C.c_int64 * (len(cfgs) * max(nsp, 1) + 1))()
    _check(lib().pic_query_sizes(arr, len(cfgs), C.byref(out), seg), "pic_query_sizes")
    return out, [int(v) for v in seg]


def pic_query_sizes_rc(cfgs: Sequence[pic_config]) -> int:
    """Return code of pic_query_sizes (for validation tests)."""
    arr = (pic_config * max(len(cfgs), 1))(*cfgs)
    out = pic_sizes()
    return int(lib().pic_query_sizes(arr, len(cfgs), C.byref(out), None))


def pic_init(cfgs: Sequence[pic_config], bufs: pic_buffers, stream: int, flags: int = 0):
    arr = (pic_config * len(cfgs))(*cfgs)
    ctx = C.c_void_p()
    _check(lib().pic_init(arr, len(cfgs), C.byref(bufs), C.c_void_p(stream), flags,
                          C.byref(ctx)), "pic_init")
    return ctx


def pic_init_static(cfgs: Sequence[pic_config], bufs: pic_buffers, stream: int, flags: int = 0):
    """pic_init with the library's static workspace (bufs.work must be NULL)."""
    arr = (pic_config * len(cfgs))(*cfgs)
    ctx = C.c_void_p()
    _check(lib().pic_init_static(arr, len(cfgs), C.byref(bufs), C.c_void_p(stream), flags,
                                 C.byref(ctx)), "pic_init_static")
    return ctx


def pic_push(ctx, flags: int = 0):
    return _check(lib().pic_push(ctx, flags), "pic_push")


def pic_deposit(ctx):
    return _check(lib().pic_deposit(ctx), "pic_deposit")


def pic_field_solve(ctx):
    return _check(lib().pic_field_solve(ctx), "pic_field_solve")


def pic_mcc_collide(ctx):
    return _check(lib().pic_mcc_collide(ctx), "pic_mcc_collide")


def pic_sort(ctx):
    return _check(lib().pic_sort(ctx), "pic_sort")


def pic_step(ctx, n_steps: int, sort_every: int = 0):
    return _check(lib().pic_step(ctx, int(n_steps), int(sort_every)), "pic_step")


def pic_step_graph(ctx, n_steps: int, sort_every: int = 0):
    return _check(lib().pic_step_graph(ctx, n_steps, sort_every), "pic_step_graph")


def pic_autotune_sort(ctx, candidates: Sequence[int], trial_steps: int):
    """(best cadence, [rate per candidate])"""
    n = len(candidates)
    cand = (C.c_int * n)(*[int(v) for v in candidates])
    rates = (C.c_double * n)()
    best = C.c_int()
    _check(lib().pic_autotune_sort(ctx, cand, n, int(trial_steps), C.byref(best), rates),
           "pic_autotune_sort")
    return best.value, list(rates)


def pic_set_mover(ctx, chunks: int, blocks: int = 0):
    return _check(lib().pic_set_mover(ctx, int(chunks), int(blocks)), "pic_set_mover")


def pic_autotune(ctx, movers: Sequence, cadences: Sequence[int], trial_steps: int):
    """((chunks, blocks) of the best mover, best cadence, [rate per mover], [rate per cadence])"""
    n, m = len(movers), len(cadences)
    ch = (C.c_int * n)(*[int(a) for a, _ in movers])
    bl = (C.c_int * n)(*[int(b) for _, b in movers])
    cad = (C.c_int * m)(*[int(v) for v in cadences])
    rates = (C.c_double * (n + m))()
    bm, bc = C.c_int(), C.c_int()
    _check(lib().pic_autotune(ctx, ch, bl, n, cad, m, int(trial_steps), C.byref(bm), C.byref(bc),
                              rates), "pic_autotune")
    r = list(rates)
    return tuple(movers[bm.value]), bc.value, r[:n], r[n:]


def pic_diagnostics(ctx, n_inst: int = 1):
    """Returns (list of pic_diag, status code) -- the diagnostics are valid either way."""
    out = (pic_diag * n_inst)()
    rc = lib().pic_diagnostics(ctx, out, n_inst)
    if rc in (PIC_E_ARG, PIC_E_DEVICE):
        raise PicError(rc, "pic_diagnostics")
    return list(out), int(rc)


def pic_region(ctx, region: int):
    off = C.c_uint64()
    n = C.c_int64()
    _check(lib().pic_region(ctx, region, C.byref(off), C.byref(n)), "pic_region")
    return int(off.value), int(n.value)


def pic_destroy(ctx):
    return _check(lib().pic_destroy(ctx), "pic_destroy")


# ---------------------------------------------------------------------------
# configuration from a workload description (duck-typed: nc, bc, dx, dt, eps0,
# B0, theta, seed, species[q, m, w, kind, v_cap, T_src], mcc, source)
# ---------------------------------------------------------------------------

def make_config(wl, precision: int, capacities: Sequence[int], n_init: Sequence[int],
                next_id: int, step0: int = 0, seed: Optional[int] = None) -> pic_config:
    c = pic_config()
    c.nc, c.bc, c.nsp, c.precision = wl.nc, wl.bc, len(wl.species), precision
    c.mcc_on = 1 if getattr(wl, "mcc", None) is not None else 0
    c.source_on = 1 if getattr(wl, "source", False) else 0
    c.seed = int(wl.seed if seed is None else seed)
    c.dx, c.dt, c.eps0 = wl.dx, wl.dt, wl.eps0
    c.B0, c.theta = wl.B0, wl.theta
    for k, s in enumerate(wl.species):
        sp = c.sp[k]
        sp.q, sp.m, sp.w, sp.kind = s.q, s.m, s.w, s.kind
        sp.nstep = int(getattr(s, "nstep", 1))
        sp.capacity = int(capacities[k])
        sp.n_init = int(n_init[k])
        sp.v_cap = getattr(s, "v_cap", 0.0)
        sp.T_src = getattr(s, "T_src", 0.0)
        sp.T_init = getattr(s, "T", 0.0)
    if c.mcc_on:
        m = wl.mcc
        c.n_n, c.T_n, c.sig_el, c.sig_iz, c.E_iz, c.sig_cx = (m.n_n, m.T_n, m.sig_el, m.sig_iz,
                                                              m.E_iz, m.sig_cx)
        c.sig_ex, c.E_ex = getattr(m, "sig_ex", 0.0), getattr(m, "E_ex", 0.0)
        c.xs_flags = PIC_XS_IZ_RATE if getattr(m, "iz_const_rate", False) else 0
    c.next_id = int(next_id)
    c.step0 = int(step0)
    c.init_amp = float(getattr(wl, "perturb_amp", 0.0))
    c.init_mode = int(getattr(wl, "perturb_mode", 1))
    c.init_opts = ((PIC_INIT_OPT_QUIET if getattr(wl, "quiet", False) else 0)
                   | (PIC_INIT_OPT_PAIR if getattr(wl, "pair_start", False) else 0))
    c.smooth_passes = int(getattr(wl, "smooth_passes", 0))
    c.field_off = 1 if getattr(wl, "field_off", False) else 0
    return c


class PicSim:
    """Device buffers (torch tensors) plus a libpic context for n_inst instances.

    ``states[i][k]`` is the initial state of species k of instance i in the
    storage form of ``precision``: for PIC_FP32 an object with cell (int32),
    f (float32), vx, vy, vz (float32) and id (uint64) arrays; for PIC_FP64 x
    (float64), vx, vy, vz (float64) and id.
    """

    def __init__(self, workloads, states, precision: int, capacities=None, flags: int = 0,
                 next_ids=None, step0: int = 0, device: str = "cuda", static_work: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpic needs a ROCm GPU; none is visible")
        self.torch = torch
        if not isinstance(workloads, (list, tuple)):
            workloads, states = [workloads], [states]
            if capacities is not None:
                capacities = [capacities]
        drawn = bool(flags & PIC_INIT_DEVICE)
        if drawn:
            # the device draws the initial particles: only their counts are needed here
            states = [None] * len(workloads)
        elif any(st is None for st in states):
            raise ValueError("an initial state is needed unless PIC_INIT_DEVICE is set")
        self.n_inst = len(workloads)
        self.precision = precision
        self.workloads = list(workloads)
        self.nsp = len(workloads[0].species)
        cfgs = []
        for i, (wl, st) in enumerate(zip(workloads, states)):
            if drawn:
                n_init = [int(round(sp.ppc * wl.nc)) for sp in wl.species]
            else:
                n_init = [int(s.id.shape[0]) for s in st]
            caps = capacities[i] if capacities is not None else [
                max(1, int(math.ceil(n * sp.cap_factor)) + 1024) for n, sp in zip(n_init, wl.species)]
            nid = next_ids[i] if next_ids is not None else int(sum(n_init))
            cfgs.append(make_config(wl, precision, caps, n_init, nid, step0))
        self.cfgs = cfgs
        sizes, seg_base = pic_query_sizes(cfgs)
        self.sizes, self.seg_base = sizes, seg_base
        n = sizes.n_slots
        fdt = torch.float64 if precision == PIC_FP64 else torch.float32
        dev = torch.device(device)
        self.x = [torch.zeros(n, dtype=fdt, device=dev) for _ in range(2)]
        self.cell = [torch.zeros(n if precision == PIC_FP32 else 1, dtype=torch.int32, device=dev)
                     for _ in range(2)]
        self.vx = [torch.zeros(n, dtype=fdt, device=dev) for _ in range(2)]
        self.vy = [torch.zeros(n, dtype=fdt, device=dev) for _ in range(2)]
        self.vz = [torch.zeros(n, dtype=fdt, device=dev) for _ in range(2)]
        # particle ids as two 32-bit words (int32 tensors holding the uint32 bits)
        self.id_lo = [torch.zeros(n, dtype=torch.int32, device=dev) for _ in range(2)]
        self.id_hi = [torch.zeros(n, dtype=torch.int32, device=dev) for _ in range(2)]
        # static_work: the context uses libpic's static workspace (pic_init_static)
        self.static_work = static_work
        self.work = None if static_work else torch.zeros(int(sizes.work_bytes), dtype=torch.uint8,
                                                         device=dev)
        # upload the initial state into set 0
        for i, st in enumerate(states):
            if st is None:
                continue
            for k, s in enumerate(st):
                b = seg_base[i * self.nsp + k]
                m = int(s.id.shape[0])
                if m == 0:
                    continue
                if precision == PIC_FP32:
                    self.x[0][b:b + m] = torch.from_numpy(np.ascontiguousarray(s.f, np.float32))
                    self.cell[0][b:b + m] = torch.from_numpy(np.ascontiguousarray(s.cell, np.int32))
                else:
                    self.x[0][b:b + m] = torch.from_numpy(np.ascontiguousarray(s.x, np.float64))
                npdt = np.float64 if precision == PIC_FP64 else np.float32
                self.vx[0][b:b + m] = torch.from_numpy(np.ascontiguousarray(s.vx, npdt))
                self.vy[0][b:b + m] = torch.from_numpy(np.ascontiguousarray(s.vy, npdt))
                self.vz[0][b:b + m] = torch.from_numpy(np.ascontiguousarray(s.vz, npdt))
                ids = np.ascontiguousarray(s.id, np.uint64)
                self.id_lo[0][b:b + m] = torch.from_numpy(
                    (ids & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32))
                self.id_hi[0][b:b + m] = torch.from_numpy((ids >> np.uint64(32)).astype(np.uint32).view(np.int32))
        bufs = pic_buffers()
        for b in range(2):
            bufs.x[b] = self.x[b].data_ptr()
            bufs.cell[b] = self.cell[b].data_ptr() if precision == PIC_FP32 else None
            bufs.vx[b] = self.vx[b].data_ptr()
            bufs.vy[b] = self.vy[b].data_ptr()
            bufs.vz[b] = self.vz[b].data_ptr()
            bufs.id_lo[b] = self.id_lo[b].data_ptr()
            bufs.id_hi[b] = self.id_hi[b].data_ptr()
        bufs.work = None if static_work else self.work.data_ptr()
        self.bufs = bufs
        self.stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        init = pic_init_static if static_work else pic_init
        self.ctx = init(cfgs, bufs, self.stream.cuda_stream, flags)

    # -- phases -------------------------------------------------------------
    def push(self, flags: int = 0):
        pic_push(self.ctx, flags)

    def deposit(self):
        pic_deposit(self.ctx)

    def field_solve(self):
        pic_field_solve(self.ctx)

    def mcc_collide(self):
        pic_mcc_collide(self.ctx)

    def sort(self):
        pic_sort(self.ctx)

    def step(self, n: int = 1, sort_every: int = 0):
        pic_step(self.ctx, n, sort_every)

    def step_graph(self, n: int = 1, sort_every: int = 0):
        pic_step_graph(self.ctx, n, sort_every)

    def autotune_sort(self, candidates=(5, 10, 20, 40, 80), trial_steps: int = 80):
        return pic_autotune_sort(self.ctx, candidates, trial_steps)

    def set_mover(self, chunks: int, blocks: int = 0):
        pic_set_mover(self.ctx, chunks, blocks)

    def autotune(self, movers, cadences=(5, 10, 20, 40, 80), trial_steps: int = 80):
        return pic_autotune(self.ctx, movers, cadences, trial_steps)

    def diagnostics(self):
        return pic_diagnostics(self.ctx, self.n_inst)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self.torch.cuda.synchronize()
            pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- views ----------------------------------------------------------------
    def region(self, region: int, dtype):
        """A torch view of a workspace region."""
        if self.work is None:
            raise RuntimeError("the static workspace of pic_init_static is not addressable")
        off, n = pic_region(self.ctx, region)
        esz = self.torch.empty(0, dtype=dtype).element_size()
        return self.work[off:off + n * esz].view(dtype)

    def grid(self, region: int, inst: int = 0):
        """Numpy copy of a grid region for one instance ([nsp][nc+1] or [nc+1])."""
        torch = self.torch
        dt = {PIC_R_DEPOSIT: torch.int64, PIC_R_RHO: torch.float64, PIC_R_PHI: torch.float64,
              PIC_R_EFIELD: torch.float64, PIC_R_ACC64: torch.float64,
              PIC_R_ACC32: torch.float32, PIC_R_CELL_OFFSETS: torch.int32,
              PIC_R_NEUTRAL_DENSITY: torch.float64}[region]
        torch.cuda.synchronize()
        a = self.region(region, dt).cpu().numpy()
        if region == PIC_R_DEPOSIT:
            a = a.view(np.uint64)
        if region == PIC_R_CELL_OFFSETS:
            a = a.view(np.uint32)
        G = int(self.sizes.n_nodes)
        nb = self.node_base()
        lo, hi = nb[inst], nb[inst + 1]
        if region in (PIC_R_DEPOSIT, PIC_R_ACC64, PIC_R_ACC32, PIC_R_CELL_OFFSETS):
            return a.reshape(self.nsp, G)[:, lo:hi].copy()
        return a[lo:hi].copy()

    def set_acc(self, acc64_list, inst: int = 0):
        """Overwrite the grid acceleration of one instance (tests)."""
        torch = self.torch
        G = int(self.sizes.n_nodes)
        nb = self.node_base()
        lo, hi = nb[inst], nb[inst + 1]
        a64 = self.region(PIC_R_ACC64, torch.float64).view(-1, G)
        a32 = self.region(PIC_R_ACC32, torch.float32).view(-1, G)
        for k, a in enumerate(acc64_list):
            t = torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(a64.device)
            a64[k, lo:hi] = t
            a32[k, lo:hi] = t.to(torch.float32)
        torch.cuda.synchronize()

    def node_base(self):
        torch = self.torch
        off, n = pic_region(self.ctx, PIC_R_NODE_BASE)
        return self.work[off:off + 8 * n].view(torch.int64).cpu().numpy()

    def _ids(self, buf: int, sl=slice(None)):
        lo = self.id_lo[buf][sl].cpu().numpy().view(np.uint32).astype(np.uint64)
        hi = self.id_hi[buf][sl].cpu().numpy().view(np.uint32).astype(np.uint64)
        return lo | (hi << np.uint64(32))

    def ids(self, buf: int, index=None):
        """Numpy uint64 ids of buffer set `buf`: every slot, or the slots a
        slice or an index tensor (on the device) selects."""
        return self._ids(buf, slice(None) if index is None else index)

    def state(self, k: int, inst: int = 0, live_only: bool = True):
        """Numpy copy of species k of instance i from the current set: a dict
        with x (float64 position in cells), vx, vy, vz (float64), id (uint64)
        and, for the FP32 form, cell and f."""
        torch = self.torch
        d, _ = self.diagnostics()
        cur = d[inst].cur_set
        n = int(d[inst].n_slots_used[k])
        b = self.seg_base[inst * self.nsp + k]
        sl = slice(b, b + n)
        out = {}
        vx = self.vx[cur][sl].cpu().numpy().astype(np.float64)
        vy = self.vy[cur][sl].cpu().numpy().astype(np.float64)
        vz = self.vz[cur][sl].cpu().numpy().astype(np.float64)
        ids = self._ids(cur, sl)
        if self.precision == PIC_FP32:
            cell = self.cell[cur][sl].cpu().numpy()
            f = self.x[cur][sl].cpu().numpy()
            live = cell >= 0
            x = cell.astype(np.float64) + f.astype(np.float64)
            out.update(cell=cell, f=f)
        else:
            x = self.x[cur][sl].cpu().numpy()
            live = x >= 0
        out.update(x=x, vx=vx, vy=vy, vz=vz, id=ids, live=live)
        if live_only:
            out = {key: (v[live] if isinstance(v, np.ndarray) and v.shape[:1] == live.shape else v)
                   for key, v in out.items()}
        return out
