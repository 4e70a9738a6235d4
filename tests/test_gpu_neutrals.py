"""GPU parity of the kinetic-neutral path (the paper's Table 1 case, Sec. 3.4:
electrons, D+ ions and ballistic D atoms, no field solver, elastic,
excitation and ionisation consuming atoms) through the C ABI.

Bars:
  * FP64 form: identical process counts (candidates, elastic, excitation,
    ionisation, consumed atoms, untargeted events), identical ids of every
    species (which atoms were consumed included), positions within 1e-9
    cells and velocities within 1e-9 v_th (the pushes are bit-exact; the
    collision kinematics agree to rounding of sqrt/log/sincos), and the node
    density of the atoms bit-exact (same integer deposit, same formula);
  * FP32 form: the ledger exactly (every ionisation consumed an atom or is
    counted untargeted; atoms + ions and electrons - ions conserved) and the
    process counts within 5 sigma of the FP64 oracle's;
  * full size (3e7 particles, FP32, drawn on the device): the decay law's
    logistic closed form for a constant rate coefficient within 5 sigma, the
    ledger exactly.
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pin
from gpu_common import FP32, FP64, P, build_pair, flush, gpu_state, oracle_state

pytestmark = pytest.mark.gpu


def table1_small(nc=200, ppc=60, ppc_n=80, seed=41, nu_dt=0.05, rate=False, n_n=4e21,
                 field_off=True, shares=(0.5, 0.2, 0.3)):
    """A Table 1 system of 10 um cells whose electron-atom processes are scaled
    so that nu_max dt = nu_dt (shares: elastic, excitation, ionisation)."""
    base = pin.table1(nc=nc, ppc=ppc, L=nc * 1e-5, seed=seed)
    e = base.species[0]
    sig = nu_dt / (n_n * e.v_cap * base.dt)
    mcc = pin.MCC(n_n=n_n, T_n=pin.EV, sig_el=shares[0] * sig, sig_ex=shares[1] * sig,
                  E_ex=10.2 * pin.EV, sig_iz=shares[2] * sig, E_iz=13.6 * pin.EV, sig_cx=0.0,
                  iz_const_rate=rate)
    wl = base.replace(mcc=mcc, field_off=field_off)
    wl.species[2].ppc = ppc_n
    return wl


def caps_for(wl, st):
    n = [s.n for s in st]
    room = 2 * n[2] + 1024
    return [n[0] + room, n[1] + room, n[2] + 1024]


def _counts(d):
    return (d.n_candidates, d.n_elastic, d.n_excite, d.n_ionize, d.n_consumed, d.n_iz_untargeted)


def _orc_counts(c):
    return (c.n_candidates, c.n_elastic, c.n_excite, c.n_ionize, c.n_consumed, c.n_iz_untargeted)


def _compare_fp64(sim, orc, wl, inst=0, d=None):
    if d is None:
        d, rc = sim.diagnostics()
        assert rc == 0, rc
    d = d[inst]
    assert _counts(d) == _orc_counts(orc.counters), (_counts(d), _orc_counts(orc.counters))
    vth = wl.vth_hat(wl.species[0])
    for k in range(3):
        g = gpu_state(sim, k) if inst == 0 else None
        if g is None:
            from gpu_common import by_id
            g = by_id(sim.state(k, inst=inst))
        o = oracle_state(orc, k)
        assert np.array_equal(g["id"], o["id"]), f"species {k}: ids differ"
        assert np.max(np.abs(g["x"] - o["x"]), initial=0.0) <= 1e-9
        for f in ("vx", "vy", "vz"):
            assert np.max(np.abs(g[f] - o[f]), initial=0.0) <= 1e-9 * vth


@pytest.mark.parametrize("sort_every", [0, 10], ids=["unsorted", "sort10"])
@pytest.mark.parametrize("rate", [False, True], ids=["sigma", "rate"])
def test_table1_fp64_matches_the_oracle(sort_every, rate):
    """30 steps; without a sort the atoms of a cell are found by scanning the
    species, with one through the cell offsets of the last sort."""
    wl = table1_small(rate=rate)
    st = pin.initial_state(wl)
    flush(f"table1 fp64 sort_every={sort_every} rate={rate}")
    flags = P.PIC_INIT_SORT if sort_every else 0
    sim, orc, ost = build_pair(wl, FP64, caps=caps_for(wl, st), flags=flags, state=st)
    # the atom density of the initial state, bit-exact
    orc.deposit()
    orc.field()
    assert np.array_equal(sim.grid(P.PIC_R_NEUTRAL_DENSITY), orc.nn)
    orc = oracle.OracleSim(wl, ost, caps=caps_for(wl, st))
    sim.step(30, sort_every=sort_every)
    orc.step(30)
    c = orc.counters
    assert c.n_ionize > 30 and c.n_excite > 30 and c.n_elastic > 30 and c.n_consumed > 30
    _compare_fp64(sim, orc, wl)
    # the atom density after the last step
    orc.deposit()
    orc.field()
    assert np.array_equal(sim.grid(P.PIC_R_NEUTRAL_DENSITY), orc.nn)
    # no field: E = phi = 0 on the GPU
    assert np.all(sim.grid(P.PIC_R_EFIELD) == 0.0) and np.all(sim.grid(P.PIC_R_PHI) == 0.0)
    sim.close()


def test_crowded_cells_fp64():
    """Few cells, few atoms, strong ionisation: several events per cell per
    step, cells running out of atoms (untargeted events)."""
    wl = table1_small(nc=16, ppc=200, ppc_n=6, nu_dt=0.3, shares=(0.0, 0.0, 1.0), rate=True,
                      n_n=2e20, seed=43)
    st = pin.initial_state(wl)
    flush("table1 crowded cells fp64")
    sim, orc, ost = build_pair(wl, FP64, caps=caps_for(wl, st), flags=P.PIC_INIT_SORT, state=st)
    sim.step(6, sort_every=3)
    orc.step(6)
    c = orc.counters
    assert c.n_consumed > 20 and c.n_iz_untargeted > 0
    _compare_fp64(sim, orc, wl)
    sim.close()


def test_field_on_and_off_instances_in_one_context_fp64():
    """Two kinetic-neutral instances, one without the field solve (Table 1)
    and one periodic with it, each against its own oracle."""
    wls = [table1_small(nc=150, seed=44), table1_small(nc=230, seed=45, field_off=False)]
    states = [pin.initial_state(w) for w in wls]
    caps = [caps_for(w, s) for w, s in zip(wls, states)]
    flush("table1 mixed field on/off fp64")
    sim = P.PicSim(wls, states, FP64, capacities=caps, flags=P.PIC_INIT_SORT)
    sim.step(20, sort_every=10)
    d, rc = sim.diagnostics()
    assert rc == 0
    for i, (w, s) in enumerate(zip(wls, states)):
        orc = oracle.OracleSim(w, s, caps=caps[i], inst=i)
        orc.step(20)
        _compare_fp64(sim, orc, w, inst=i, d=d)
    E1 = sim.grid(P.PIC_R_EFIELD, inst=1)
    assert np.all(sim.grid(P.PIC_R_EFIELD, inst=0) == 0.0) and np.any(E1 != 0.0)
    sim.close()


def test_table1_fp32_ledger_and_counts():
    wl = table1_small(nc=400, ppc=80, ppc_n=80, seed=46)
    st = pin.initial_state(wl)
    flush("table1 fp32")
    sim, orc, ost = build_pair(wl, FP32, caps=caps_for(wl, st), flags=P.PIC_INIT_SORT, state=st)
    sim.step(40, sort_every=20)
    orc.step(40)
    d, rc = sim.diagnostics()
    assert rc == 0
    d = d[0]
    n0 = [s.n for s in ost]
    assert d.n_consumed + d.n_iz_untargeted == d.n_ionize
    assert d.n_live[2] == n0[2] - d.n_consumed
    assert d.n_live[0] == n0[0] + d.n_ionize and d.n_live[1] == n0[1] + d.n_ionize
    c = orc.counters
    for g, o in zip(_counts(d)[:5], _orc_counts(c)[:5]):
        assert abs(g - o) <= 5 * math.sqrt(2 * max(o, 1)) + 2, (_counts(d), _orc_counts(c))
    sim.close()


def test_full_size_table1_decay_law_fp32():
    """The Table 1 workload at full size (100,000 cells, 100 particles per cell
    per species, 3e7 particles, FP32, drawn on the device and sorted), with the
    ionisation replaced by a constant rate coefficient large enough to deplete
    the gas in 150 steps: the atom count follows the logistic solution of
    dn/dt = -n n_e R within 5 sigma; every ionisation consumed an atom."""
    wl = pin.table1()
    e = wl.species[0]
    n_n = 2e21
    nu_dt = 2e-3
    sig = nu_dt / (n_n * e.v_cap * wl.dt)
    wl = wl.replace(mcc=pin.MCC(n_n=n_n, T_n=pin.EV, sig_el=0.0, sig_iz=sig, E_iz=0.0,
                                sig_cx=0.0, iz_const_rate=True))
    n = int(round(100 * wl.nc))
    caps = [n + n // 2 + 1024, n + n // 2 + 1024, n + 1024]
    flush("full size table1: draw on the device")
    sim = P.PicSim(wl, None, FP32, capacities=caps, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_SORT)
    P_c = -math.expm1(-nu_dt)
    a = P_c * wl.species[2].w / (wl.nc * wl.dx * n_n)
    Ne0 = N0 = n
    C = Ne0 + N0
    s_done = 0
    for s_end in (50, 100, 150):
        flush(f"full size table1: steps to {s_end}")
        sim.step(s_end - s_done, sort_every=20)
        s_done = s_end
        d, rc = sim.diagnostics()
        assert rc == 0, rc
        d = d[0]
        N = d.n_live[2]
        closed = C * N0 / (N0 + (C - N0) * math.exp(a * C * s_end))
        assert abs(N - closed) < 5 * math.sqrt(N0 - closed) + 1e-4 * N0, (s_end, N, closed)
        assert d.n_consumed == d.n_ionize and d.n_iz_untargeted == 0
        assert d.n_live[0] == Ne0 + (N0 - N) and d.n_live[1] == n + (N0 - N)
    assert N0 - N > 0.1 * N0
    sim.close()


@pytest.mark.parametrize("case", ["walls_field_on", "subcycled_atoms"])
def test_table1_variants_fp64(case):
    """Kinetic atoms between absorbing walls with the field solved (particles
    lost to the walls), and atoms pushed every 4 steps
    (the reach of the cell-offset search takes the subcycle into account)."""
    if case == "walls_field_on":
        wl = table1_small(nc=180, seed=47, field_off=False).replace(bc=pin.BC_ABSORB)
    else:
        wl = table1_small(nc=160, seed=48)
        wl.species[2].nstep = 4
    st = pin.initial_state(wl)
    flush(f"table1 variant {case} fp64")
    sim, orc, ost = build_pair(wl, FP64, caps=caps_for(wl, st), flags=P.PIC_INIT_SORT, state=st)
    sim.step(25, sort_every=10)
    orc.step(25)
    c = orc.counters
    assert c.n_consumed > 20
    if case == "walls_field_on":
        assert sum(c.absorbed_total[0][w] for w in range(2)) > 0  # electrons reached the walls
    _compare_fp64(sim, orc, wl)
    sim.close()


def test_many_kinetic_instances_fp64():
    """350 small Table 1 instances (1050 segments, beyond the LDS tables):
    every instance's counts against its own oracle, ids for a sample."""
    wls = [table1_small(nc=30 + (i % 9) * 4, ppc=24, ppc_n=24, seed=100 + i) for i in range(350)]
    states = [pin.initial_state(w) for w in wls]
    caps = [caps_for(w, s) for w, s in zip(wls, states)]
    flush("350 kinetic instances, 1050 segments")
    sim = P.PicSim(wls, states, FP64, capacities=caps, flags=P.PIC_INIT_SORT)
    sim.step(10, sort_every=5)
    d, rc = sim.diagnostics()
    assert rc == 0
    consumed = 0
    for i, (w, s) in enumerate(zip(wls, states)):
        orc = oracle.OracleSim(w, s, caps=caps[i], inst=i)
        orc.step(10)
        if i % 25 == 0:
            _compare_fp64(sim, orc, w, inst=i, d=d)
        else:
            assert _counts(d[i]) == _orc_counts(orc.counters), i
        consumed += orc.counters.n_consumed
    assert consumed > 100
    sim.close()
