"""The shared overflow lists of the collision step against the oracle.

The mover writes each collision candidate into its block's own region of the
candidate list; a wave whose part of the region is full appends the rest to a
shared overflow list, which the collide blocks split among themselves.  The
collide kernel likewise writes ionisation events into per-block regions with
a shared overflow list.  Both overflows are rare on the benchmark workloads,
so these cases force them from the host with the workload's shape:

* candidates: a gas so dense that every particle is a candidate (P_null = 1
  for electrons, 0.996 for ions), no ionisation, no source, and exactly as
  many particles as slots, 1.5 tiles per block of the persistent grid: the
  blocks that own two tiles get about 510 candidates per wave against parts
  of 384 (1,024 blocks in both forms);
* ionisation events: the same dense gas with an ionisation cross section ten
  times the elastic one, so that a collide block meets about 250 ionisations
  against an event region of 84.

One step on the oracle's field, by the separate phase calls and by the step
driver (whose movers collide their own regions and leave only the overflow
list to the collide kernel), then counts, ids, positions and velocities
against the oracle (FP64 identical counts and ids; FP32 within the FP32
tolerance of the one-step test)."""
import numpy as np
import pytest

import pic_inputs as pin
from gpu_common import FP32, FP64, P, build_pair, flush, gpu_state, oracle_state

pytestmark = pytest.mark.gpu

TILE = 1024                  # particles per mover tile
GRID = {FP32: 1024, FP64: 1024}  # persistent grid of the movers, blocks


def _one_step(wl, prec, caps, fused):
    """One step on the oracle's field.  fused: the step driver's path (each
    mover block collides its own region, the collide kernel only the
    overflow list); else pic_push then pic_mcc_collide."""
    sim, orc, ost = build_pair(wl, prec, caps=caps, flags=P.PIC_INIT_NO_FIELD)
    orc.deposit()
    orc.field()
    acc = [a.copy() for a in orc.acc]
    orc.push()
    orc.walls()
    orc.mcc()
    orc.source()
    sim.set_acc(acc)
    if fused:
        sim.step(1)
    else:
        sim.push()
        sim.mcc_collide()
    d, rc = sim.diagnostics()
    return sim, orc, d[0], rc


def _compare(sim, orc, d, wl, prec):
    c = orc.counters
    if prec == FP64:
        assert d.n_candidates == c.n_candidates
        assert (d.n_elastic, d.n_ionize, d.n_cx) == (c.n_elastic, c.n_ionize, c.n_cx)
        assert d.n_source == c.n_source and d.next_id == c.next_id
    else:
        assert d.n_candidates == c.n_candidates  # the test is integer, on ids and step only
        for a, b in ((d.n_elastic, c.n_elastic), (d.n_ionize, c.n_ionize), (d.n_cx, c.n_cx)):
            assert abs(a - b) <= max(4, 1e-4 * b)
    tol = 1e-12 if prec == FP64 else 2e-5
    for k, s in enumerate(wl.species):
        g, o = gpu_state(sim, k), oracle_state(orc, k)
        if prec == FP64:
            assert np.array_equal(g["id"], o["id"]), k
            gi = oi = np.arange(g["id"].size)
        else:
            _, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
            assert g["id"].size - gi.size <= 16 and o["id"].size - oi.size <= 16
        vth = wl.vth_hat(s)
        assert np.max(np.abs(g["x"][gi] - o["x"][oi])) <= (0 if prec == FP64 else 1e-5), k
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f][gi] - o[f][oi]) / np.maximum(np.abs(o[f][oi]), vth)
            # an FP32 velocity near a process boundary may take the other process
            bad = np.count_nonzero(err > tol)
            assert bad <= (0 if prec == FP64 else 16), (k, f, bad, float(np.max(err)))


@pytest.mark.parametrize("fused", [False, True], ids=["phases", "step"])
@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_candidate_overflow_list(prec, fused):
    nc, ppc = 1024, 576
    n = nc * ppc                       # 576 full tiles per species
    wl = pin.bounded_mcc(nc=nc, ppc=ppc, seed=61, source=False)
    wl.mcc.n_n = 1e27
    wl.mcc.sig_iz = 0.0
    flush(f"candidate overflow prec={prec} fused={fused}")
    # the shape forces the overflow: 1.5 tiles per block, every particle a candidate
    n_tiles = 2 * n // TILE
    grid = min(n_tiles, GRID[prec])
    assert n_tiles == 1152 and n_tiles > grid
    sim, orc, d, rc = _one_step(wl, prec, [n, n], fused)
    T = [orc.candidate_threshold(k) for k in range(2)]
    expect = n * (T[0] + T[1]) / 2 ** 32
    cand_q = max(1024, -(-(int(1.25 * expect / grid) + 64) // 64) * 64)
    per_wave_two_tiles = (TILE // 4) * (T[0] + T[1]) / 2 ** 32
    assert T[0] == 2 ** 32 and per_wave_two_tiles > cand_q / 4 + 8
    assert rc == 0 and d.status == 0, f"status {d.status:#x}"
    assert orc.counters.n_candidates > 0.99 * 2 * n
    _compare(sim, orc, d, wl, prec)
    sim.close()


@pytest.mark.parametrize("fused", [False, True], ids=["phases", "step"])
@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_ionisation_event_overflow_list(prec, fused):
    nc, ppc = 512, 100
    wl = pin.bounded_mcc(nc=nc, ppc=ppc, seed=62)
    wl.mcc.n_n = 1e27
    wl.mcc.sig_iz = 10 * wl.mcc.sig_el
    flush(f"ionisation event overflow prec={prec} fused={fused}")
    n = nc * ppc
    caps = [3 * n, 3 * n]
    sim, orc, d, rc = _one_step(wl, prec, caps, fused)
    n_tiles = 2 * (-(-3 * n // TILE))
    grid = min(n_tiles, GRID[prec])
    T = [orc.candidate_threshold(k) for k in range(2)]
    expect = 3 * n * (T[0] + T[1]) / 2 ** 32
    cand_q = max(1024, -(-(int(1.25 * expect / grid) + 64) // 64) * 64)
    ev_q = max(32, cand_q // 16)
    busy = -(-n // TILE)               # blocks whose tile holds electrons
    assert orc.counters.n_ionize > 2 * busy * ev_q
    assert rc == 0 and d.status == 0, f"status {d.status:#x}"
    _compare(sim, orc, d, wl, prec)
    sim.close()
