"""Seeded synthetic inputs for the 1D3V electrostatic PIC-MCC step.

This module is the only code shared by the GPU library's tests/bench and the
CPU oracle.  It builds workload descriptions (grid, species, collision and
source parameters in SI units) and seeded initial particle states.  It holds
none of the method's arithmetic: no deposition, field solve, push, collision
or diagnostic is computed here.

Units of the particle state handed to both sides:
  * position ``x`` in cell units, domain [0, nc)  (x = X / dx),
  * velocity ``v`` in cells per step               (v = V * dt / dx).
These are the in-cell coordinates and the ``x += nstep*vx`` advance of the
paper's mover (Sec. 2 and the moveb listing in Sec. 6), with nstep = 1.

Workloads:
  * ``langmuir``   periodic electron plasma on a neutralising background,
                   512 cells, 100 particles/cell, plasma units (eps0 = 1,
                   omega_p = 1, q/m = -1), lambda_D = 0.5 dx, omega_p dt = 0.1,
                   mode-1 density perturbation 1e-3; ``quiet=True`` gives the
                   cold lattice start used for the Langmuir-frequency pin.
  * ``bounded``    1D3V plasma between grounded absorbing walls, electrons and
                   ions (m_i/m_e = 1836, T_i = T_e = 20 eV, n0 = 1e21 m^-3 as in
                   the paper's Table 1), lambda_De = 0.5 dx, omega_pe dt = 0.1,
                   B at 45 deg to the wall normal with omega_ce dt = 0.2, pair
                   source on.  Default 8192 cells x 200 particles/cell/species.
  * ``bounded_mcc`` the same plus null-collision MCC against a neutral
                   background (n_n = 1e3 n0, T_n = 1 eV), 100,000 cells x 100
                   particles/cell/species, cell sort every 20 steps.
  * ``table1``     the paper's Table 1 test case (periodic, unmagnetised, no
                   field solve, 100,000 cells, 1 m): electrons, D+ ions and
                   kinetic D neutrals, elastic, excitation and ionisation.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# CODATA 2018 exact / recommended values (SI)
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
EPS0_SI = 8.8541878128e-12
EV = E_CHARGE  # 1 eV in joules

KIND_ELECTRON = 0
KIND_ION = 1
KIND_NEUTRAL = 2   # kinetic neutral atom (q = 0): moved ballistically, consumed by ionisation

BC_PERIODIC = 0
BC_ABSORB = 1


@dataclass
class Species:
    name: str
    kind: int          # KIND_ELECTRON / KIND_ION
    q: float           # charge [C] (plasma units for the Langmuir case)
    m: float           # mass [kg]
    w: float           # real particles per macro-particle per unit area [m^-2]
    ppc: float         # initial macro-particles per cell
    T: float           # initial temperature [J] (0 = cold)
    T_src: float = 0.0  # temperature of source-born particles [J]
    v_cap: float = 0.0  # speed bounding the null-collision frequency [m/s]
    cap_factor: float = 1.5  # capacity / initial count
    nstep: int = 1      # pushed every nstep steps over nstep dt (subcycling)


@dataclass
class MCC:
    n_n: float          # neutral density [m^-3]
    T_n: float          # neutral temperature [J]
    sig_el: float       # electron-neutral elastic cross section [m^2]
    sig_iz: float       # electron-impact ionisation cross section [m^2]
    E_iz: float         # ionisation threshold [J]
    sig_cx: float       # ion-neutral charge exchange cross section [m^2]
    sig_ex: float = 0.0  # electron-impact excitation cross section [m^2]
    E_ex: float = 0.0    # excitation threshold [J]
    iz_const_rate: bool = False  # ionisation rate coefficient sig_iz v_cap, constant in |v|


@dataclass
class Workload:
    name: str
    nc: int
    bc: int
    dx: float
    dt: float
    eps0: float
    species: List[Species]
    B0: float = 0.0
    theta: float = 0.0          # angle of B to the wall normal (x axis), in the x-y plane
    mcc: Optional[MCC] = None
    source: bool = False
    seed: int = 1
    sort_every: int = 0
    n_steps: int = 200
    perturb_amp: float = 0.0    # mode-1 density perturbation (Langmuir case)
    perturb_mode: int = 1
    quiet: bool = False         # lattice positions instead of random ones
    pair_start: bool = False    # every ion starts at an electron's position (neutral start)
    state_seed: Optional[int] = None  # seed of the initial-state generator (default: seed)
    smooth_passes: int = 0      # binomial density-smoother passes before the field solve
    field_off: bool = False     # no field solve (E = 0), as in the paper's Table 1 case

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    @property
    def n_particles(self) -> int:
        return int(sum(round(s.ppc * self.nc) for s in self.species))

    def vth_hat(self, s: Species) -> float:
        """Thermal speed sqrt(T/m) expressed in cells per step."""
        return math.sqrt(s.T / s.m) * self.dt / self.dx if s.T > 0 else 0.0


# ---------------------------------------------------------------------------
# workload builders
# ---------------------------------------------------------------------------

def langmuir(nc: int = 512, ppc: int = 100, quiet: bool = False, seed: int = 1,
             perturb_amp: float = 1e-3, n_steps: int = 200,
             cold: Optional[bool] = None) -> Workload:
    """Periodic electron plasma on an immobile neutralising background.

    Plasma units: eps0 = 1, electron charge density -1, q/m = -1, so
    omega_p = 1.  L = 1, dx = 1/nc, lambda_D = 0.5 dx, dt = 0.1 / omega_p.
    """
    L = 1.0
    dx = L / nc
    n_e = nc * ppc
    # n0 * L = total electrons per unit area = n_e * w  with n0 = 1
    w = 1.0 * L / n_e
    vth = 0.5 * dx  # lambda_D * omega_p
    cold = quiet if cold is None else cold
    T = 0.0 if cold else vth * vth * 1.0  # T = m vth^2 with m = 1
    e = Species("e", KIND_ELECTRON, q=-1.0, m=1.0, w=w, ppc=ppc, T=T, cap_factor=1.0)
    return Workload(name="langmuir" + ("_quiet" if quiet else ""), nc=nc, bc=BC_PERIODIC,
                    dx=dx, dt=0.1, eps0=1.0, species=[e], seed=seed, n_steps=n_steps,
                    perturb_amp=perturb_amp, quiet=quiet)


def _bounded_plasma_scales(n0: float, Te: float):
    lam_d = math.sqrt(EPS0_SI * Te / (n0 * E_CHARGE ** 2))
    w_pe = math.sqrt(n0 * E_CHARGE ** 2 / (EPS0_SI * M_ELECTRON))
    return lam_d, w_pe


def bounded(nc: int = 8192, ppc: float = 200, seed: int = 2, n_steps: int = 10000,
            mass_ratio: float = 1836.0, Te_eV: float = 20.0, n0: float = 1e21,
            theta_deg: float = 45.0, wce_dt: float = 0.2, wpe_dt: float = 0.1,
            source: bool = True, sort_every: int = 20, cap_factor: float = 1.5) -> Workload:
    """Bounded 1D3V plasma between two grounded absorbing walls."""
    Te = Te_eV * EV
    lam_d, w_pe = _bounded_plasma_scales(n0, Te)
    dx = lam_d / 0.5  # lambda_De = 0.5 dx
    dt = wpe_dt / w_pe
    m_i = mass_ratio * M_ELECTRON
    w = n0 * dx / ppc
    B0 = wce_dt * M_ELECTRON / (E_CHARGE * dt) if wce_dt > 0 else 0.0
    e = Species("e", KIND_ELECTRON, q=-E_CHARGE, m=M_ELECTRON, w=w, ppc=ppc, T=Te,
                T_src=Te, cap_factor=cap_factor)
    i = Species("i", KIND_ION, q=E_CHARGE, m=m_i, w=w, ppc=ppc, T=Te, T_src=Te,
                cap_factor=cap_factor)
    return Workload(name="bounded", nc=nc, bc=BC_ABSORB, dx=dx, dt=dt, eps0=EPS0_SI,
                    species=[e, i], B0=B0, theta=math.radians(theta_deg), source=source,
                    seed=seed, sort_every=sort_every, n_steps=n_steps, pair_start=True)


def default_mcc(n0: float = 1e21) -> MCC:
    """Constant cross sections (builder's defaults; no data in the paper)."""
    return MCC(n_n=1e3 * n0, T_n=1.0 * EV, sig_el=1e-19, sig_iz=1e-21, E_iz=15.0 * EV,
               sig_cx=5e-19)


def bounded_mcc(nc: int = 100_000, ppc: float = 100, seed: int = 3, n_steps: int = 10000,
                sort_every: int = 20, cap_factor: float = 1.5, v_cap_eV: float = 200.0,
                **kw) -> Workload:
    """Bounded plasma plus null-collision MCC against a uniform neutral gas."""
    wl = bounded(nc=nc, ppc=ppc, seed=seed, n_steps=n_steps, sort_every=sort_every,
                 cap_factor=cap_factor, **kw)
    mcc = default_mcc()
    for s in wl.species:
        s.v_cap = math.sqrt(2.0 * v_cap_eV * EV / s.m)
    return wl.replace(name="bounded_mcc", mcc=mcc)


def batched(n_inst: int = 256, seed: int = 4, nc_min: int = 256, nc_ratio: float = 64.0,
            ppc_range=(50.0, 400.0), theta_deg_max: float = 85.0,
            wpe_dt_range=(0.05, 0.2)) -> List[Workload]:
    """Independent bounded MCC instances of mixed shape, batched in one context.

    Per instance i: nc = round(nc_min * nc_ratio^U) (log-uniform), total
    particles per cell ~ U[ppc_range] split evenly between the two species,
    B at theta ~ U[0, theta_deg_max] degrees, omega_pe dt ~ U[wpe_dt_range].
    All instances share the generator seed `seed`; the collision generator
    of instance i is keyed with seed_hi xor i, and its initial state is drawn
    from its own stream (seed, i).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_inst):
        nc = int(round(nc_min * nc_ratio ** rng.random()))
        ppc_total = ppc_range[0] + (ppc_range[1] - ppc_range[0]) * rng.random()
        theta = theta_deg_max * rng.random()
        wpe_dt = wpe_dt_range[0] + (wpe_dt_range[1] - wpe_dt_range[0]) * rng.random()
        wl = bounded_mcc(nc=nc, ppc=0.5 * ppc_total, seed=seed, theta_deg=theta,
                         wpe_dt=wpe_dt, sort_every=0)
        out.append(wl.replace(name=f"batched[{i}]", state_seed=seed * 1_000_003 + i))
    return out


def table1(nc: int = 100_000, ppc: float = 100, seed: int = 6, n_steps: int = 200_000,
           L: float = 1.0, sort_every: int = 20, cap_factor: float = 1.25,
           mcc: Optional[MCC] = None, v_cap_eV: float = 400.0) -> Workload:
    """The paper's Table 1 test case (Sec. 3.4): an initially uniform hot
    plasma (electrons and D+ ions, 1e21 m^-3, 20 eV) in a uniform deuterium
    gas of kinetic neutral atoms (1e21 m^-3, 1 eV), periodic, unmagnetised,
    no field solver; electron-neutral elastic, excitation and ionisation
    collisions; 1 m, 100,000 cells, 100 particles/cell/species, dt = 4e-14 s,
    200,000 steps.

    The paper gives no cross sections.  The defaults are constant stand-ins
    of the right size for deuterium: elastic 1e-19 m^2, excitation 5e-21 m^2
    above 10.2 eV, ionisation 5e-21 m^2 above 13.6 eV.  n_n is the bound of
    the local neutral density used by the null-collision test (2 n0).
    """
    n0 = 1e21
    dx = L / nc
    w = n0 * dx / ppc
    Te = 20.0 * EV
    m_d = 2.0 * 1836.15267343 * M_ELECTRON       # deuteron (the D+ ion)
    e = Species("e", KIND_ELECTRON, q=-E_CHARGE, m=M_ELECTRON, w=w, ppc=ppc, T=Te,
                cap_factor=cap_factor)
    i = Species("D+", KIND_ION, q=E_CHARGE, m=m_d, w=w, ppc=ppc, T=Te, cap_factor=cap_factor)
    n = Species("D", KIND_NEUTRAL, q=0.0, m=m_d + M_ELECTRON, w=w, ppc=ppc, T=1.0 * EV,
                cap_factor=1.0)
    for s in (e, i, n):
        s.v_cap = math.sqrt(2.0 * v_cap_eV * EV / s.m)
    if mcc is None:
        mcc = MCC(n_n=2.0 * n0, T_n=1.0 * EV, sig_el=1e-19, sig_iz=5e-21, E_iz=13.6 * EV,
                  sig_cx=0.0, sig_ex=5e-21, E_ex=10.2 * EV)
    return Workload(name="table1", nc=nc, bc=BC_PERIODIC, dx=dx, dt=4e-14, eps0=EPS0_SI,
                    species=[e, i, n], mcc=mcc, seed=seed, n_steps=n_steps,
                    sort_every=sort_every, field_off=True)


# ---------------------------------------------------------------------------
# initial states
# ---------------------------------------------------------------------------

@dataclass
class SpeciesState:
    x: np.ndarray    # float64, cell units
    vx: np.ndarray   # float64, cells/step
    vy: np.ndarray
    vz: np.ndarray
    id: np.ndarray   # uint64

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def initial_state(wl: Workload) -> List[SpeciesState]:
    """Seeded initial particles, one SpeciesState per species.

    Positions are uniform in [0, nc) (or a lattice for ``quiet``), then, if
    ``perturb_amp`` is set, displaced by (A/k) sin(k x) with k = 2 pi m / nc,
    which gives a density modulation of relative amplitude A in mode m.
    With ``pair_start`` every species after the first reuses the first
    species' positions (equal counts), so the initial charge density is zero
    everywhere: independent uniform positions would leave a random-walk charge
    imbalance whose 1D field grows with the square root of the number of cells.
    Velocities are Maxwellian with sqrt(T/m) per component.  Ids are
    0..N_0-1 for species 0, then the next block for species 1, and so on.
    """
    rng = np.random.Generator(np.random.PCG64(wl.seed if wl.state_seed is None else wl.state_seed))
    out: List[SpeciesState] = []
    next_id = 0
    nc = wl.nc
    first_x = None
    for s in wl.species:
        n = int(round(s.ppc * nc))
        if wl.pair_start and first_x is not None and first_x.shape[0] == n:
            x = first_x.copy()
        elif wl.quiet:
            x = (np.arange(n, dtype=np.float64) + 0.5) * (nc / n)
        else:
            x = rng.random(n, dtype=np.float64) * nc
        if wl.perturb_amp != 0.0 and s.kind == KIND_ELECTRON:
            k = 2.0 * math.pi * wl.perturb_mode / nc
            x = x + (wl.perturb_amp / k) * np.sin(k * x)
            if wl.bc == BC_PERIODIC:
                x = np.mod(x, nc)
        # keep every position strictly inside [0, nc)
        x = np.where(x >= nc, np.nextafter(float(nc), 0.0), x)
        x = np.where(x < 0.0, 0.0, x)
        if first_x is None:
            first_x = x
        vt = wl.vth_hat(s)
        if vt > 0.0:
            v = rng.standard_normal((3, n)) * vt
        else:
            v = np.zeros((3, n))
        ids = np.arange(next_id, next_id + n, dtype=np.uint64)
        next_id += n
        out.append(SpeciesState(x=x, vx=v[0].copy(), vy=v[1].copy(), vz=v[2].copy(), id=ids))
    return out


def capacities(wl: Workload, state: List[SpeciesState]) -> List[int]:
    caps = []
    for s, st in zip(wl.species, state):
        caps.append(int(math.ceil(st.n * s.cap_factor)) + 1024)
    return caps


# ---------------------------------------------------------------------------
# FP32 form of a state: (cell int32, in-cell offset f float32, v float32)
# ---------------------------------------------------------------------------

@dataclass
class SpeciesStateF32:
    cell: np.ndarray  # int32
    f: np.ndarray     # float32 in [0, 1)
    vx: np.ndarray    # float32
    vy: np.ndarray
    vz: np.ndarray
    id: np.ndarray    # uint64

    def as_f64(self) -> SpeciesState:
        """The exact FP64 value of this FP32-form state (every conversion is exact)."""
        return SpeciesState(x=self.cell.astype(np.float64) + self.f.astype(np.float64),
                            vx=self.vx.astype(np.float64), vy=self.vy.astype(np.float64),
                            vz=self.vz.astype(np.float64), id=self.id.copy())


def to_fp32_form(state: List[SpeciesState], nc: int) -> List[SpeciesStateF32]:
    """Round a FP64 state to the FP32 storage form.

    The in-cell offset is rounded to float32; if that rounds up to 1.0 the
    particle is moved to offset 0 of the next cell (or, in the last cell,
    kept at the largest float32 below 1).
    """
    out = []
    below_one = np.float32(1.0 - 2.0 ** -24)
    for st in state:
        cell = np.floor(st.x).astype(np.int64)
        f = (st.x - cell).astype(np.float32)
        up = f >= np.float32(1.0)
        last = up & (cell + 1 >= nc)
        cell = np.where(up & ~last, cell + 1, cell)
        f = np.where(up & ~last, np.float32(0.0), f)
        f = np.where(last, below_one, f).astype(np.float32)
        out.append(SpeciesStateF32(cell=cell.astype(np.int32), f=f,
                                   vx=st.vx.astype(np.float32), vy=st.vy.astype(np.float32),
                                   vz=st.vz.astype(np.float32), id=st.id.copy()))
    return out
