"""GPU checks of properties that hold at any size, edge cases of the ABI on
the device, and the full-size bench workload on sampled particles.

* sort: the output is a permutation of the live particles (multiset of
  (id, state) preserved), cells are non-decreasing in every segment, and the
  cell offsets equal the scan of the per-cell counts;
* deposit: every live particle contributes exactly 2^32 after every step;
* ids stay unique; run-to-run results are identical as sets keyed by id;
* graph replay: steps replayed from a captured HIP graph (with eager work and
  synchronisation between the replays, and a start that is not aligned with
  the sort period) equal the same steps enqueued one by one, bit for bit;
* resume: k steps, a dump of the live particles, a new context from the dump
  and k more steps equal 2k steps in one context, bit for bit;
* edge cases: an empty species, ragged counts, a capacity overflow, a
  particle at |vx| >= 1 cell/step, non-finite or out-of-range uploads;
* full size (100,000 cells, 2e7 particles, FP32 form): the bit-exact deposit
  of the whole state and one step of a sample of particles against the
  oracle.
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pin
from gpu_common import FP32, FP64, P, build_pair, by_id, flush, gpu_state, oracle_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_sort_is_a_permutation_by_cell(prec):
    wl = pin.bounded_mcc(nc=600, ppc=45, seed=31)
    flush(f"sort invariants prec={prec}")
    sim, orc, ost = build_pair(wl, prec)
    sim.step(7)  # particles drift, some are absorbed, pairs are appended
    before = [gpu_state(sim, k) for k in range(2)]
    sim.sort()
    d, rc = sim.diagnostics()
    assert rc == 0 and d[0].cur_set == 1
    offs = sim.grid(P.PIC_R_CELL_OFFSETS)
    for k in range(2):
        raw = sim.state(k, live_only=False)
        assert np.all(raw["live"]), "the sort drops absorbed particles"
        cells = np.floor(raw["x"]).astype(np.int64)
        assert np.all(np.diff(cells) >= 0), "cells not sorted"
        after = by_id(raw)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(after[f], before[k][f])
        counts = np.bincount(cells, minlength=wl.nc)
        assert np.array_equal(offs[k][:wl.nc + 1].astype(np.int64),
                              np.concatenate([[0], np.cumsum(counts)]))
        assert d[0].n_slots_used[k] == d[0].n_live[k] == after["id"].size
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_charge_identity_every_step_and_unique_ids(prec):
    wl = pin.bounded_mcc(nc=333, ppc=61, seed=32)
    flush(f"charge identity prec={prec}")
    sim, orc, ost = build_pair(wl, prec)
    for s in range(25):
        sim.push()
        sim.mcc_collide()
        S = sim.grid(P.PIC_R_DEPOSIT)
        d, rc = sim.diagnostics()
        assert rc == 0
        for k in range(2):
            assert int(S[k].sum(dtype=np.uint64)) == d[0].n_live[k] * 2 ** 32
        ids = np.concatenate([gpu_state(sim, k)["id"] for k in range(2)])
        assert np.unique(ids).size == ids.size
        sim.field_solve()
        if s % 10 == 9:
            sim.sort()
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_run_to_run_identical(prec):
    wl = pin.bounded_mcc(nc=300, ppc=50, seed=33)
    flush(f"determinism prec={prec}")
    outs = []
    for _ in range(2):
        sim, orc, ost = build_pair(wl, prec)
        sim.step(30, sort_every=10)
        outs.append([gpu_state(sim, k) for k in range(2)])
        d, rc = sim.diagnostics()
        assert rc == 0
        sim.close()
    for k in range(2):
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(outs[0][k][f], outs[1][k][f])


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_graph_replays_equal_eager_steps(prec):
    wl = pin.bounded_mcc(nc=500, ppc=60, seed=39)
    wl.mcc.n_n *= 10
    flush(f"graph replay prec={prec}")
    a, _, _ = build_pair(wl, prec)
    b, _, _ = build_pair(wl, prec)
    a.step(67, sort_every=20)
    b.step_graph(7, 20)        # eager: the first sort comes after step 20
    b.step_graph(13, 20)       # eager up to the sort
    b.step_graph(20, 20)       # one replay
    d, rc = b.diagnostics()    # eager kernels and a synchronisation between replays
    assert rc == 0 and d[0].step == 40
    mid = [gpu_state(b, k) for k in range(2)]
    b.step_graph(20, 20)       # the same graph again
    d, rc = b.diagnostics()
    assert rc == 0 and d[0].step == 60 and mid[0]["id"].size > 0
    b.step_graph(7, 20)        # remainder, eager
    da, rca = a.diagnostics()
    db, rcb = b.diagnostics()
    assert rca == 0 and rcb == 0 and da[0].step == db[0].step == 67
    for f in ("n_candidates", "n_elastic", "n_ionize", "n_cx", "n_source", "next_id",
              "particle_steps"):
        assert getattr(da[0], f) == getattr(db[0], f), f
    for k in range(2):
        ga, gb = gpu_state(a, k), gpu_state(b, k)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(ga[f], gb[f]), f
    # a period that starts 7 steps into the cadence: the graph holds 13 steps,
    # the sort, then 7 more; two replays and a remainder of 5, eager
    a.step(45, sort_every=20)
    b.step_graph(45, 20)
    da, _ = a.diagnostics()
    db, rcb = b.diagnostics()
    assert rcb == 0 and da[0].step == db[0].step == 112
    for k in range(2):
        ga, gb = gpu_state(a, k), gpu_state(b, k)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(ga[f], gb[f]), f
    # without sorting: a graph of one step, replayed
    a.step(9, sort_every=0)
    b.step_graph(9, 0)
    for k in range(2):
        ga, gb = gpu_state(a, k), gpu_state(b, k)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(ga[f], gb[f]), f
    a.close()
    b.close()


def test_autotune_sort_picks_a_candidate_and_leaves_a_valid_state():
    wl = pin.bounded_mcc(nc=2000, ppc=50, seed=42)
    flush("autotune sort cadence")
    sim, _, _ = build_pair(wl, FP32)
    best, rates = sim.autotune_sort((5, 10, 20, 0), 20)
    assert best in (5, 10, 20, 0)
    assert len(rates) == 4 and all(r > 0 for r in rates)
    d, rc = sim.diagnostics()
    assert rc == 0 and d[0].step == 180  # a warm-up trial, then two rounds of four, 20 steps each
    sim.step(7, best)
    d, rc = sim.diagnostics()
    assert rc == 0 and d[0].step == 187
    for k in range(2):
        ids = gpu_state(sim, k)["id"]
        assert np.unique(ids).size == ids.size
    sim.close()


COUNTS = ("n_candidates", "n_elastic", "n_ionize", "n_cx", "n_over_cap", "n_source", "particle_steps",
          "next_id")


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_mover_shapes_give_identical_results(prec):
    """pic_set_mover: the mover in one pass of 4 chunks or two passes of 2, on
    the default grid or on twice as many blocks, switched between steps,
    computes exactly what the default computes (every particle by id, every
    counter) over 30 steps with collisions, pairs, source and sorts."""
    wl = pin.bounded_mcc(nc=2000, ppc=300, seed=44)
    wl.mcc.n_n *= 5
    flush(f"mover shapes prec={prec}")
    st64 = pin.initial_state(wl)
    state = pin.to_fp32_form(st64, wl.nc) if prec == FP32 else st64
    caps = pin.capacities(wl, st64)
    ref = P.PicSim(wl, state, prec, capacities=caps)
    nb, nmax = int(ref.sizes.mover_blocks), int(ref.sizes.mover_blocks_max)
    assert nmax > nb  # the workload has tiles for more than one residency
    ref.step(30, 10)
    d0, rc = ref.diagnostics()
    assert rc == 0
    want = [gpu_state(ref, k) for k in range(2)]
    ref.close()
    plans = [[(2, 0)], [(4, nmax)], [(2, nmax)], [(4, 0), (2, nmax), (4, 0)]]
    for plan in plans:
        sim = P.PicSim(wl, state, prec, capacities=caps)
        for i, (chunks, blocks) in enumerate(plan):
            sim.set_mover(chunks, blocks)
            sim.step(30 // len(plan), 10)
        d, rc = sim.diagnostics()
        assert rc == 0 and d[0].step == 30, plan
        for f in COUNTS:
            assert getattr(d[0], f) == getattr(d0[0], f), (plan, f)
        for k in range(2):
            g = gpu_state(sim, k)
            for f in ("id", "x", "vx", "vy", "vz"):
                assert np.array_equal(g[f], want[k][f]), (plan, k, f)
        sim.close()


def test_mover_shape_arguments_are_checked():
    wl = pin.bounded_mcc(nc=300, ppc=20, seed=45)
    sim, _, _ = build_pair(wl, FP32)
    for chunks, blocks in ((3, 0), (8, 0), (4, -1), (4, int(sim.sizes.mover_blocks_max) + 1)):
        with pytest.raises(P.PicError) as e:
            sim.set_mover(chunks, blocks)
        assert e.value.code == P.PIC_E_ARG
    sim.close()


def test_autotune_picks_a_mover_and_a_cadence():
    """pic_autotune over mover shapes, then sort cadences, on a batch of
    instances: it returns one of the candidates, leaves the context on that
    shape, and the state stays valid."""
    wls = pin.batched(n_inst=8, seed=46)
    flush("autotune mover shape and cadence")
    sim = P.PicSim(wls, [None] * len(wls), FP32, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_SORT)
    nmax = int(sim.sizes.mover_blocks_max)
    movers = [(4, 0), (2, 0), (4, nmax), (2, nmax)]
    best, cad, mrates, crates = sim.autotune(movers, (10, 20), 20)
    assert best in movers and cad in (10, 20)
    assert len(mrates) == 4 and len(crates) == 2 and all(r > 0 for r in mrates + crates)
    d, rc = sim.diagnostics()
    # shapes: a warm-up trial and two rounds of four; cadences: a warm-up and two of two (20 steps each)
    assert rc == 0 and all(x.step == 20 * (1 + 8 + 1 + 4) for x in d)
    sim.step(7, cad)
    d, rc = sim.diagnostics()
    assert rc == 0
    for i in range(len(wls)):
        for k in range(2):
            ids = sim.state(k, inst=i)["id"]
            assert np.unique(ids).size == ids.size
    sim.close()


def _dump(sim, k, prec):
    """Live particles of species k in the storage form of `prec`."""
    from types import SimpleNamespace
    st = sim.state(k)
    if prec == FP32:
        return SimpleNamespace(cell=st["cell"], f=st["f"], vx=st["vx"].astype(np.float32),
                               vy=st["vy"].astype(np.float32), vz=st["vz"].astype(np.float32),
                               id=st["id"])
    return SimpleNamespace(x=st["x"], vx=st["vx"], vy=st["vy"], vz=st["vz"], id=st["id"])


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_resume_from_a_dump_is_bit_identical(prec):
    wl = pin.bounded_mcc(nc=400, ppc=50, seed=38)
    wl.mcc.n_n *= 20
    flush(f"resume prec={prec}")
    full, _, _ = build_pair(wl, prec)
    full.step(30, sort_every=10)
    half, _, _ = build_pair(wl, prec)
    half.step(15, sort_every=10)
    d, rc = half.diagnostics()
    assert rc == 0
    dump = [_dump(half, k, prec) for k in range(2)]
    caps = [int(half.cfgs[0].sp[k].capacity) for k in range(2)]
    half.close()
    res = P.PicSim(wl, dump, prec, capacities=caps, next_ids=[int(d[0].next_id)],
                   step0=int(d[0].step))
    res.step(15, sort_every=10)
    da, rca = full.diagnostics()
    db, rcb = res.diagnostics()
    assert rca == 0 and rcb == 0
    assert da[0].step == db[0].step and da[0].next_id == db[0].next_id
    for k in range(2):
        ga, gb = gpu_state(full, k), gpu_state(res, k)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(ga[f], gb[f]), f
    full.close()
    res.close()


def test_empty_species_and_ragged_counts():
    # periodic electrons (ragged count, 211 particles) plus an ion species with no particles;
    # the neutralising background keeps the system quiet
    wl = pin.langmuir(nc=64, ppc=3.3)
    wl.species.append(pin.Species("i", pin.KIND_ION, q=1.0, m=100.0, w=wl.species[0].w, ppc=0,
                                  T=0.0))
    st = pin.initial_state(wl)
    assert st[0].n == 211 and st[1].n == 0
    flush("empty species")
    sim, orc, ost = build_pair(wl, FP64, state=st, caps=[st[0].n + 5, 8])
    sim.step(5)
    orc.step(5)
    d, rc = sim.diagnostics()
    assert rc == 0 and d[0].n_live[1] == 0
    g, o = gpu_state(sim, 0), oracle_state(orc, 0)
    assert np.array_equal(g["id"], o["id"])
    assert np.max(np.abs(g["x"] - o["x"])) <= 1e-9
    sim.close()


def test_capacity_overflow_is_flagged():
    """Source pairs that do not fit are dropped and reported, never written out of bounds."""
    wl = pin.bounded(nc=64, ppc=20, seed=35, source=True)
    st = pin.initial_state(wl)
    # ions near the walls and fast towards them: many are absorbed in the first step
    for s in st:
        s.vx[:] = np.where(s.x < 32, -0.9, 0.9)
    caps = [st[0].n, st[1].n]  # no room for the source pairs beyond the slots freed by nothing
    flush("capacity overflow")
    sim, _, _ = build_pair(wl, FP32, state=st, caps=caps)
    sim.step(2)
    d, rc = sim.diagnostics()
    assert rc == P.PIC_E_CAPACITY and (d[0].status & P.PIC_ST_CAPACITY)
    for k in range(2):
        assert d[0].n_slots_used[k] <= caps[k]
    sim.close()


def test_cfl_breach_is_flagged():
    wl = pin.bounded(nc=64, ppc=5, seed=36, source=False)
    st = pin.initial_state(wl)
    st[0].vx[3] = 1.5  # cells per step
    flush("cfl")
    sim, _, _ = build_pair(wl, FP64, state=st)
    sim.step(1)
    d, rc = sim.diagnostics()
    assert rc == P.PIC_E_CFL and (d[0].status & P.PIC_ST_CFL)
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_bad_upload_is_dropped_and_flagged(prec):
    wl = pin.bounded(nc=64, ppc=5, seed=37, source=False)
    st = pin.initial_state(wl)
    st[0].vx[1] = np.nan
    st[0].x[2] = 64.5  # outside [0, nc)
    flush(f"bad upload prec={prec}")
    sim, _, _ = build_pair(wl, prec, state=st)
    d, rc = sim.diagnostics()
    assert d[0].status & P.PIC_ST_BAD_INIT
    assert d[0].n_live[0] == st[0].n - 2
    sim.step(2)
    d, rc = sim.diagnostics()
    assert np.all(np.isfinite(gpu_state(sim, 0)["vx"]))
    sim.close()


def test_periodic_wrap_fp32_matches_oracle():
    wl = pin.langmuir(nc=128, ppc=50)
    st = pin.initial_state(wl)
    st[0].vx[:] = np.where(np.arange(st[0].n) % 2 == 0, 0.7, -0.7)  # many wall crossings
    flush("periodic wrap")
    sim, orc, ost = build_pair(wl, FP32, state=st)
    sim.step(3)
    orc.step(3)
    g, o = gpu_state(sim, 0), oracle_state(orc, 0)
    assert np.array_equal(g["id"], o["id"])
    dxw = np.abs(g["x"] - o["x"])
    dxw = np.minimum(dxw, wl.nc - dxw)  # positions on a ring
    assert np.max(dxw) <= 1e-5
    sim.close()


@pytest.mark.slow
def test_full_size_bench_workload_sampled():
    """100,000 cells, 2e7 particles: bit-exact deposit of the whole uploaded state, then
    one step of the FP32 form compared with the oracle on a sample of particles."""
    wl = pin.bounded_mcc(nc=100_000, ppc=100, seed=3, cap_factor=1.25)
    flush("full size: generate")
    st = pin.initial_state(wl)
    st32 = pin.to_fp32_form(st, wl.nc)
    caps = pin.capacities(wl, st)
    flush("full size: deposit")
    sim = P.PicSim(wl, st32, FP32, capacities=caps, flags=P.PIC_INIT_NO_FIELD)
    sim.deposit()
    S = sim.grid(P.PIC_R_DEPOSIT)
    ost = [s.as_f64() for s in st32]
    for k in range(2):
        assert np.array_equal(S[k], oracle.deposit_fixed(ost[k].x, wl.nc))
    sim.close()
    flush("full size: one step")
    sim = P.PicSim(wl, st32, FP32, capacities=caps)
    sim.push(P.PIC_PUSH_NO_DEPOSIT)
    # oracle: field of the whole state, push of a sample
    full = oracle.OracleSim(wl, ost, caps=caps)
    full.deposit()
    full.field()
    rng = np.random.default_rng(0)
    for k, s in enumerate(wl.species):
        pick = np.sort(rng.choice(ost[k].n, 20000, replace=False))
        sub = pin.SpeciesState(x=ost[k].x[pick], vx=ost[k].vx[pick], vy=ost[k].vy[pick],
                               vz=ost[k].vz[pick], id=ost[k].id[pick])
        sample_states = [sub if q == k else pin.SpeciesState(x=np.zeros(0), vx=np.zeros(0),
                                                               vy=np.zeros(0), vz=np.zeros(0),
                                                               id=np.zeros(0, np.uint64))
                         for q in range(2)]
        o = oracle.OracleSim(wl, sample_states, caps=[pick.size + 1] * 2)
        for q in range(2):
            o.acc[q][:] = full.acc[q]
        o.push()
        o.walls()
        os_ = oracle_state(o, k)
        g = gpu_state(sim, k)
        gi = np.searchsorted(g["id"], os_["id"])
        ok = (gi < g["id"].size)
        gi = np.minimum(gi, g["id"].size - 1)
        ok &= g["id"][gi] == os_["id"]
        assert ok.mean() > 0.999
        vth = wl.vth_hat(s)
        assert np.max(np.abs(g["x"][gi[ok]] - os_["x"][ok])) <= 1e-5
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f][gi[ok]] - os_[f][ok]) / np.maximum(np.abs(os_[f][ok]), vth)
            assert np.max(err) <= 1e-5
    sim.close()
