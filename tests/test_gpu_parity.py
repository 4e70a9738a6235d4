"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bars (stated per test):
  * deposition: bit-exact (integer fixed point) on the same positions;
  * charge density rho: bit-exact (same integer inputs, same FP64 formula);
  * field solve: |phi_gpu - phi_orc| <= 8 nc eps64 max|phi| (the GPU evaluates
    the Thomas recurrences as parallel scans, the oracle sequentially; both
    are within ~nc eps64 of the exact solution);
  * FP64 push on the oracle's grid acceleration: bit-exact;
  * FP32 push: position error <= 1e-5 cells, velocity error <= 1e-5 max(|v64|, v_th)
    per component (the single-step per-particle tolerance of the FP32 form).
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pin
from gpu_common import FP32, FP64, P, build_pair, by_id, flush, gpu_state, oracle_state

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -52

WORKLOADS = {
    "langmuir": lambda: pin.langmuir(),                               # 512 cells, 51,200 e
    "bounded_ragged": lambda: pin.bounded(nc=300, ppc=37.3, seed=7),  # 2 species, ragged counts
    "bounded_mcc": lambda: pin.bounded_mcc(nc=700, ppc=50, seed=8),
    # density smoother on: three passes with walls, two on a periodic grid
    "bounded_smooth3": lambda: pin.bounded(nc=300, ppc=37.3, seed=9).replace(pair_start=False,
                                                                              smooth_passes=3),
    "langmuir_smooth2": lambda: pin.langmuir(nc=256, ppc=40).replace(smooth_passes=2),
}


def _deposit_ref(orc_state, nc):
    return [oracle.deposit_fixed(s.x, nc) for s in orc_state]


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_deposit_bit_exact(name, prec):
    wl = WORKLOADS[name]()
    flush(f"deposit {name} prec={prec}")
    sim, orc, ost = build_pair(wl, prec, flags=P.PIC_INIT_NO_FIELD)
    sim.deposit()
    S = sim.grid(P.PIC_R_DEPOSIT)
    ref = _deposit_ref(ost, wl.nc)
    for k in range(len(wl.species)):
        assert np.array_equal(S[k], ref[k]), f"species {k}: max diff {np.max(np.abs(S[k].astype(np.int64) - ref[k].astype(np.int64)))}"
        assert int(S[k].sum(dtype=np.uint64)) == ost[k].n * 2 ** 32
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_field_solve(name, prec):
    wl = WORKLOADS[name]()
    flush(f"field {name} prec={prec}")
    _check_field(wl, prec)


# Grids of several field tiles (1024 nodes each): the solve's tile-level
# scans take runs of one tile per thread up to 256 tiles, of up to four in
# registers up to 1024 tiles, and longer runs read tile by tile beyond.
# (electrons and ions drawn apart, so that the charge density is not zero)
def _apart(nc, ppc, seed, **kw):
    return pin.bounded(nc=nc, ppc=ppc, seed=seed, source=False).replace(pair_start=False, **kw)


MANY_TILES = {
    "bounded_3_tiles": lambda: _apart(3000, 4, 21),
    "periodic_3_tiles": lambda: pin.langmuir(nc=3000, ppc=4, seed=22),
    "bounded_293_tiles": lambda: _apart(300_000, 1, 23),
    "periodic_293_tiles": lambda: pin.langmuir(nc=300_000, ppc=1, seed=24),
    "bounded_1075_tiles": lambda: _apart(1_100_000, 1, 25),
    "bounded_smooth2_40_tiles": lambda: _apart(40_000, 2, 26, smooth_passes=2),
}


@pytest.mark.parametrize("name", list(MANY_TILES))
def test_field_solve_many_tiles(name):
    wl = MANY_TILES[name]()
    flush(f"field {name} (nc={wl.nc})")
    _check_field(wl, FP64)


def _check_field(wl, prec):
    sim, orc, ost = build_pair(wl, prec, flags=P.PIC_INIT_NO_FIELD)
    sim.deposit()
    sim.field_solve()
    orc.deposit()
    orc.field()
    rho = sim.grid(P.PIC_R_RHO)
    assert np.array_equal(rho, orc.rho), f"rho max diff {np.max(np.abs(rho - orc.rho))}"
    phi = sim.grid(P.PIC_R_PHI)
    E = sim.grid(P.PIC_R_EFIELD)
    tol_phi = 8 * wl.nc * EPS64 * np.max(np.abs(orc.phi))
    assert np.max(np.abs(phi - orc.phi)) <= tol_phi
    tol_E = 2 * tol_phi / wl.dx + 8 * EPS64 * np.max(np.abs(orc.E))
    assert np.max(np.abs(E - orc.E)) <= tol_E
    a64 = sim.grid(P.PIC_R_ACC64)
    a32 = sim.grid(P.PIC_R_ACC32)
    for k, s in enumerate(wl.species):
        C = (s.q / s.m) * (wl.dt * wl.dt / wl.dx)
        assert np.max(np.abs(a64[k] - orc.acc[k])) <= abs(C) * tol_E * 1.01
        assert np.max(np.abs(a32[k] - orc.acc[k])) <= abs(C) * tol_E + 2 ** -23 * np.max(np.abs(orc.acc[k]))
    # the deposit is consumed
    assert int(sim.grid(P.PIC_R_DEPOSIT).sum()) == 0
    sim.close()


def _oracle_one_push(orc):
    orc.deposit()
    orc.field()
    acc = [a.copy() for a in orc.acc]
    orc.push()
    orc.walls()
    return acc


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_push_fp64_bit_exact_on_oracle_field(name):
    """Given the oracle's grid acceleration, one FP64 push reproduces the oracle bit for bit,
    and so does the fused deposit of the new positions."""
    wl = WORKLOADS[name]()
    flush(f"push fp64 {name}")
    sim, orc, ost = build_pair(wl, FP64, flags=P.PIC_INIT_NO_FIELD)
    acc = _oracle_one_push(orc)
    sim.set_acc(acc)
    sim.push()
    for k in range(len(wl.species)):
        g, o = gpu_state(sim, k), oracle_state(orc, k)
        assert np.array_equal(g["id"], o["id"])
        for f in ("x", "vx", "vy", "vz"):
            assert np.array_equal(g[f], o[f]), f"{f}: max diff {np.max(np.abs(g[f] - o[f]))}"
    S = sim.grid(P.PIC_R_DEPOSIT)
    orc.deposit()
    for k in range(len(wl.species)):
        assert np.array_equal(S[k], orc.S[k])
    sim.close()


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_push_fp32_tolerance(name):
    wl = WORKLOADS[name]()
    flush(f"push fp32 {name}")
    sim, orc, ost = build_pair(wl, FP32, flags=P.PIC_INIT_NO_FIELD)
    acc = _oracle_one_push(orc)
    sim.set_acc(acc)
    sim.push()
    for k, s in enumerate(wl.species):
        g, o = gpu_state(sim, k), oracle_state(orc, k)
        # absorption decisions can differ only for particles within rounding of a wall
        common, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
        only = np.setxor1d(g["id"], o["id"])
        if only.size:
            ox = np.concatenate([ost[k].x[np.isin(ost[k].id, only)]])
            assert only.size <= 2, f"{only.size} particles absorbed on one side only"
        vth = max(wl.vth_hat(s), 1e-30)
        dx_ = np.abs(g["x"][gi] - o["x"][oi])
        assert np.max(dx_) <= 1e-5, f"position error {np.max(dx_)}"
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f][gi] - o[f][oi]) / np.maximum(np.abs(o[f][oi]), vth)
            assert np.max(err) <= 1e-5, f"{f} relative error {np.max(err)}"
    # fused deposit: every live particle contributes exactly 2^32
    S = sim.grid(P.PIC_R_DEPOSIT)
    d, _ = sim.diagnostics()
    for k in range(len(wl.species)):
        assert int(S[k].sum(dtype=np.uint64)) == int(np.sum(gpu_state(sim, k)["id"].size)) * 2 ** 32
    sim.close()


@pytest.mark.parametrize("nc", [300, 300_000], ids=["deposit_in_l2", "deposit_beyond_l2"])
def test_push_fp32_fused_deposit_matches_the_deposit_kernel(nc):
    """The FP32 mover's fused deposit flushes its window after the next pass's
    loads when the deposit array fits in 4 MiB (2 species x 301 nodes) and at
    the end of each pass otherwise (2 x 300,001 nodes x 8 B = 4.8 MB): either
    way it equals, node for node, the deposit kernel's of the positions it
    wrote (that kernel is bit-exact against the oracle in
    test_deposit_bit_exact)."""
    wl = pin.bounded(nc=nc, ppc=37.3 if nc < 1000 else 2, seed=31)
    flush(f"fused deposit fp32 nc={nc}")
    sim = P.PicSim(wl, None, FP32, flags=P.PIC_INIT_DEVICE)
    sim.push()
    S1 = sim.grid(P.PIC_R_DEPOSIT).astype(np.uint64)
    sim.deposit()  # adds the same positions again
    S2 = sim.grid(P.PIC_R_DEPOSIT).astype(np.uint64) - S1
    d, _ = sim.diagnostics()
    for k in range(2):
        assert np.array_equal(S1[k], S2[k])
        assert int(S1[k].sum(dtype=np.uint64)) == int(d[0].n_live[k]) * 2 ** 32
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_mcc_one_step(prec):
    """Push + collisions + ionisation pairs + source for one step, on the oracle's field."""
    wl = pin.bounded_mcc(nc=400, ppc=80, seed=11)
    # a denser gas so that every process fires many times in one step
    wl.mcc.n_n *= 20
    flush(f"mcc one step prec={prec}")
    sim, orc, ost = build_pair(wl, prec, flags=P.PIC_INIT_NO_FIELD)
    orc.deposit()
    orc.field()
    acc = [a.copy() for a in orc.acc]
    orc.push()
    orc.walls()
    orc.mcc()
    orc.source()
    sim.set_acc(acc)
    sim.push()
    sim.mcc_collide()
    d, rc = sim.diagnostics()
    d = d[0]
    c = orc.counters
    assert rc == 0 and d.status == 0
    if prec == FP64:
        assert d.n_candidates == c.n_candidates
        assert d.n_elastic == c.n_elastic and d.n_ionize == c.n_ionize and d.n_cx == c.n_cx
        assert d.n_source == c.n_source
    else:
        assert abs(d.n_candidates - c.n_candidates) <= 2
        for a, b in ((d.n_elastic, c.n_elastic), (d.n_ionize, c.n_ionize), (d.n_cx, c.n_cx)):
            assert abs(a - b) <= 2
    assert c.n_elastic > 100 and c.n_ionize > 5 and c.n_cx > 20
    assert d.next_id == c.next_id if prec == FP64 else abs(int(d.next_id) - int(c.next_id)) <= 8
    tol = 1e-12 if prec == FP64 else 2e-5
    for k, s in enumerate(wl.species):
        g, o = gpu_state(sim, k), oracle_state(orc, k)
        if prec == FP64:
            assert np.array_equal(g["id"], o["id"])
            gi = oi = np.arange(g["id"].size)
        else:
            _, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
            assert g["id"].size - gi.size <= 8 and o["id"].size - oi.size <= 8
        vth = wl.vth_hat(s)
        assert np.max(np.abs(g["x"][gi] - o["x"][oi])) <= (0 if prec == FP64 else 1e-5)
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f][gi] - o[f][oi]) / np.maximum(np.abs(o[f][oi]), vth)
            assert np.max(err) <= tol, f"species {k} {f}: {np.max(err)}"
    sim.close()


def _check_momentum(d, od, wl, rel):
    """Momentum per species and component against the oracle's, within rel of
    the sum of |m w V| (bounded by sqrt(2 m w N KE))."""
    for k, s in enumerate(wl.species):
        scale = math.sqrt(2.0 * s.m * s.w * od.n[k] * od.ke[k])
        for c in range(3):
            assert abs(d.mom[k][c] - od.mom[k][c]) <= rel * scale, (k, c, d.mom[k][c], od.mom[k][c])


def test_langmuir_fp64_200_steps():
    """Whole steps (push, close of step, field solve) for the plain-method workload."""
    wl = pin.langmuir()
    flush("langmuir fp64 200 steps")
    sim, orc, ost = build_pair(wl, FP64)
    sim.step(200)
    orc.step(200)
    # the GPU solves the field at x^200 at the end of step 199; bring the oracle's field there
    orc.deposit()
    orc.field()
    d, rc = sim.diagnostics()
    od = orc.diagnostics()
    assert rc == 0 and d[0].step == 200 and d[0].n_live[0] == 51200
    g, o = gpu_state(sim, 0), oracle_state(orc, 0)
    assert np.array_equal(g["id"], o["id"])
    # trajectories start identical and drift apart only through rounding of the field solve
    assert np.max(np.abs(g["x"] - o["x"])) <= 1e-8
    assert np.max(np.abs(g["vx"] - o["vx"])) <= 1e-10
    assert abs(d[0].ke[0] / od.ke[0] - 1) <= 1e-10
    _check_momentum(d[0], od, wl, 1e-10)
    assert abs(d[0].field_energy / od.field_energy - 1) <= 1e-6
    assert d[0].particle_steps == 200 * 51200
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_bounded_mcc_steps_with_sort(prec):
    """60 whole steps with walls, collisions, source and a sort every 20 steps."""
    wl = pin.bounded_mcc(nc=256, ppc=40, seed=12)
    flush(f"bounded mcc 60 steps prec={prec}")
    sim, orc, ost = build_pair(wl, prec)
    sim.step(60, sort_every=20)
    orc.step(60)
    d, rc = sim.diagnostics()
    d = d[0]
    c = orc.counters
    od = orc.diagnostics()
    assert rc == 0 and d.status == 0 and d.step == 60
    for k in range(2):
        ids = gpu_state(sim, k)["id"]
        assert np.unique(ids).size == ids.size
        if prec == FP64:
            assert d.n_live[k] == od.n[k]
            assert np.array_equal(ids, oracle_state(orc, k)["id"])
        else:
            assert abs(d.n_live[k] - od.n[k]) <= max(3, 0.002 * od.n[k])
    if prec == FP64:
        assert d.n_ionize == c.n_ionize and d.n_source == c.n_source
        for k in range(2):
            g, o = gpu_state(sim, k), oracle_state(orc, k)
            assert np.max(np.abs(g["x"] - o["x"])) <= 1e-7
            assert abs(d.ke[k] / od.ke[k] - 1) <= 1e-9
        _check_momentum(d, od, wl, 1e-9)
    else:
        for k in range(2):
            assert abs(d.ke[k] / od.ke[k] - 1) <= 5e-3
    sim.close()


def test_batched_instances_match_the_oracle_one_by_one():
    """Independent instances of mixed shape in one context (FP64): each one,
    collision generator keyed by its instance index, against its own oracle."""
    wls = pin.batched(n_inst=5, seed=41, nc_min=64, nc_ratio=8.0, ppc_range=(40.0, 120.0))
    states = [pin.initial_state(w) for w in wls]
    caps = [pin.capacities(w, s) for w, s in zip(wls, states)]
    flush("batched instances: " + ", ".join(f"{w.nc}x{w.species[0].ppc:.1f}" for w in wls))
    sim = P.PicSim(wls, states, FP64, capacities=caps)
    sim.step(40, sort_every=20)
    d, rc = sim.diagnostics()
    assert rc == 0
    for i, (w, s) in enumerate(zip(wls, states)):
        orc = oracle.OracleSim(w, s, caps=caps[i], inst=i)
        orc.step(40)
        od = orc.diagnostics()
        assert d[i].step == 40
        assert d[i].n_ionize == orc.counters.n_ionize and d[i].n_source == orc.counters.n_source
        for k in range(2):
            g = by_id(sim.state(k, inst=i))
            o = oracle_state(orc, k)
            assert d[i].n_live[k] == od.n[k]
            assert np.array_equal(g["id"], o["id"])
            assert np.max(np.abs(g["x"] - o["x"])) <= 1e-7
            assert abs(d[i].ke[k] / od.ke[k] - 1) <= 1e-9
    sim.close()


# ---------------------------------------------------------------------------
# the drawn initial state (PIC_INIT_DEVICE) against the oracle's generator
# ---------------------------------------------------------------------------
INIT_WORKLOADS = {
    "bounded_mcc_pair": lambda: pin.bounded_mcc(nc=700, ppc=50, seed=51),
    "bounded_indep_ragged": lambda: pin.bounded_mcc(nc=300, ppc=37.3, seed=52).replace(pair_start=False),
    "langmuir_perturbed": lambda: pin.langmuir(perturb_amp=1e-2),
    "langmuir_quiet_cold": lambda: pin.langmuir(nc=128, ppc=20, quiet=True, perturb_amp=1e-3),
}


def _check_drawn(sim, wl, o, prec, inst=0):
    exact_x = wl.perturb_amp == 0.0
    for k, s in enumerate(wl.species):
        g = sim.state(k, inst=inst)  # slot p holds particle p
        assert np.array_equal(g["id"], o[k].id)
        vth = wl.vth_hat(s)
        if prec == FP64:
            if exact_x:
                assert np.array_equal(g["x"], o[k].x)
            else:
                assert np.max(np.abs(g["x"] - o[k].x)) <= 1e-12 * wl.nc
            for f in ("vx", "vy", "vz"):
                assert np.max(np.abs(g[f] - getattr(o[k], f))) <= 1e-13 * vth
        else:
            ref = pin.to_fp32_form([o[k]], wl.nc)[0]
            if exact_x:
                assert np.array_equal(g["cell"], ref.cell) and np.array_equal(g["f"], ref.f)
            else:
                assert np.max(np.abs(g["x"] - ref.as_f64().x)) <= 1e-6
            for f in ("vx", "vy", "vz"):
                r = getattr(ref, f).astype(np.float64)
                assert np.max(np.abs(g[f] - r)) <= 2.0 ** -23 * np.max(np.abs(r)) + 1e-30


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("name", list(INIT_WORKLOADS))
def test_drawn_initial_state_matches_the_oracle(name, prec):
    """Positions bit-exact (no perturbation; else within rounding of sin), velocities
    within a few ulps (the device's log/sin/cos against the host's), ids exact, and the
    deposit of the drawn state bit-exact against the oracle's."""
    wl = INIT_WORKLOADS[name]()
    flush(f"drawn init {name} prec={prec}")
    sim = P.PicSim(wl, None, prec, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_NO_FIELD)
    d, rc = sim.diagnostics()
    assert rc == 0 and d[0].status == 0
    o = oracle.init_state(wl)
    _check_drawn(sim, wl, o, prec)
    if wl.perturb_amp == 0.0:
        sim.deposit()
        S = sim.grid(P.PIC_R_DEPOSIT)
        ref = oracle.init_deposit(wl, fp32_form=(prec == FP32))
        for k in range(len(wl.species)):
            assert np.array_equal(S[k], ref[k])
    sim.close()


def test_drawn_initial_state_of_batched_instances():
    wls = pin.batched(n_inst=4, seed=53, nc_min=64, nc_ratio=8.0, ppc_range=(40.0, 120.0))
    flush("drawn init batched")
    sim = P.PicSim(wls, [None] * len(wls), FP64, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_NO_FIELD)
    for i, w in enumerate(wls):
        _check_drawn(sim, w, oracle.init_state(w, inst=i), FP64, inst=i)
    sim.close()


def test_drawn_state_rejects_ids_below_the_initial_count():
    wl = pin.bounded_mcc(nc=64, ppc=10, seed=54)
    with pytest.raises(P.PicError):
        P.PicSim(wl, None, FP32, flags=P.PIC_INIT_DEVICE, next_ids=[10])


def _sampled_slots(sim, k, idx):
    """The FP32-form state of slots seg_base + idx of species k (buffer set 0)."""
    import torch
    b = int(sim.seg_base[k])
    ii = torch.from_numpy(np.asarray(idx, np.int64) + b).to(sim.x[0].device)
    cell = sim.cell[0][ii].cpu().numpy()
    f = sim.x[0][ii].cpu().numpy()
    out = {"x": cell.astype(np.float64) + f.astype(np.float64), "cell": cell}
    for name in ("vx", "vy", "vz"):
        out[name] = getattr(sim, name)[0][ii].cpu().numpy().astype(np.float64)
    out["id"] = sim.ids(0, ii)
    return out


@pytest.mark.slow
def test_full_size_1e6_cells_drawn_state_sampled():
    """1,000,000 cells and 200 particles per cell per species (4e8 particles), FP32
    form, drawn on the device.  Bit-exact: the sampled initial particles and the
    deposit of all 4e8.  Then rho bit-exact, phi/E within the solve's rounding, and
    one push of 20,000 sampled particles per species against the oracle's push on the
    oracle's own field (independent positions, so the field is not zero)."""
    wl = pin.bounded_mcc(nc=1_000_000, ppc=200, seed=5).replace(pair_start=False)
    n = int(round(200 * wl.nc))
    caps = [n + n // 20 + 1024] * 2
    flush("full size 1e6 cells: draw on the device")
    sim = P.PicSim(wl, None, FP32, capacities=caps, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_NO_FIELD)
    d, rc = sim.diagnostics()
    assert rc == 0 and d[0].n_live[0] == n and d[0].n_live[1] == n
    rng = np.random.default_rng(5)
    pick = [np.sort(rng.choice(n, 20000, replace=False)) for _ in range(2)]
    o = oracle.init_state(wl, select=pick)
    for k in range(2):
        g = _sampled_slots(sim, k, pick[k])
        ref = pin.to_fp32_form([o[k]], wl.nc)[0]
        assert np.array_equal(g["id"], o[k].id)
        assert np.array_equal(g["x"], ref.as_f64().x)
    flush("full size 1e6 cells: deposit (oracle: 4e8 particles on one core)")
    sim.deposit()
    S = sim.grid(P.PIC_R_DEPOSIT)
    S_ref = oracle.init_deposit(wl, fp32_form=True)
    for k in range(2):
        assert np.array_equal(S[k], S_ref[k])
    flush("full size 1e6 cells: field")
    sim.field_solve()
    empty = [pin.SpeciesState(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0),
                              id=np.zeros(0, np.uint64)) for _ in range(2)]
    full = oracle.OracleSim(wl, empty, caps=[1, 1])
    for k in range(2):
        full.S[k][:] = S_ref[k]
    full.field()
    assert np.array_equal(sim.grid(P.PIC_R_RHO), full.rho)
    tol_phi = 8 * wl.nc * EPS64 * np.max(np.abs(full.phi))
    assert np.max(np.abs(sim.grid(P.PIC_R_PHI) - full.phi)) <= tol_phi
    flush("full size 1e6 cells: one push of the sample")
    sim.push(P.PIC_PUSH_NO_DEPOSIT)
    for k, s in enumerate(wl.species):
        sub = pin.SpeciesState(x=pin.to_fp32_form([o[k]], wl.nc)[0].as_f64().x,
                               vx=o[k].vx.astype(np.float32).astype(np.float64),
                               vy=o[k].vy.astype(np.float32).astype(np.float64),
                               vz=o[k].vz.astype(np.float32).astype(np.float64), id=o[k].id)
        states = [sub if q == k else empty[q] for q in range(2)]
        one = oracle.OracleSim(wl, states, caps=[pick[k].size + 1] * 2)
        for q in range(2):
            one.acc[q][:] = full.acc[q]
        one.push()
        one.walls()
        os_ = oracle_state(one, k)
        g = _sampled_slots(sim, k, pick[k])
        live = g["cell"] >= 0
        # absorption can differ only for a particle within rounding of a wall
        common, gi, oi = np.intersect1d(g["id"][live], os_["id"], return_indices=True)
        assert np.setxor1d(g["id"][live], os_["id"]).size <= 2
        vth = wl.vth_hat(s)
        gx = g["x"][live][gi]
        assert np.max(np.abs(gx - os_["x"][oi])) <= 1e-5
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f][live][gi] - os_[f][oi]) / np.maximum(np.abs(os_[f][oi]), vth)
            assert np.max(err) <= 1e-5
    sim.close()


@pytest.mark.slow
def test_full_size_batched_256_instances_drawn_sampled():
    """The 256-instance batched workload at full size (2.5e8 particles, FP32 form, drawn
    on the device, sorted at init), in the configuration the benchmark runs: for three
    instances, sampled drawn particles exact, the deposit of every particle of the
    instance bit-exact, rho bit-exact and phi within the solve's rounding; the
    diagnostics of every instance report all its particles."""
    import torch
    wls = pin.batched(n_inst=256, seed=4)
    flush("batched 256: draw on the device")
    sim = P.PicSim(wls, [None] * len(wls), FP32, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_NO_FIELD)
    d, rc = sim.diagnostics()
    assert rc == 0
    for i, w in enumerate(wls):
        for k, s in enumerate(w.species):
            assert d[i].n_live[k] == int(round(s.ppc * w.nc))
    sim.deposit()
    S = [sim.grid(P.PIC_R_DEPOSIT, inst=i) for i in (0, 97, 255)]
    sim.field_solve()
    rng = np.random.default_rng(44)
    for n_i, i in enumerate((0, 97, 255)):
        w = wls[i]
        flush(f"batched 256: instance {i} ({w.nc} cells)")
        n = [int(round(s.ppc * w.nc)) for s in w.species]
        pick = [np.sort(rng.choice(n[k], min(n[k], 2000), replace=False)) for k in range(2)]
        o = oracle.init_state(w, inst=i, select=pick)
        for k in range(2):
            b = int(sim.seg_base[i * 2 + k])
            ii = torch.from_numpy(pick[k].astype(np.int64) + b).to(sim.x[0].device)
            x = sim.cell[0][ii].cpu().numpy().astype(np.float64) + sim.x[0][ii].cpu().numpy().astype(np.float64)
            ref = pin.to_fp32_form([o[k]], w.nc)[0]
            assert np.array_equal(x, ref.as_f64().x)
            assert np.array_equal(sim.ids(0, ii), o[k].id)
        S_ref = oracle.init_deposit(w, inst=i, fp32_form=True)
        for k in range(2):
            assert np.array_equal(S[n_i][k], S_ref[k])
        empty = [pin.SpeciesState(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0),
                                  id=np.zeros(0, np.uint64)) for _ in range(2)]
        orc = oracle.OracleSim(w, empty, caps=[1, 1], inst=i)
        for k in range(2):
            orc.S[k][:] = S_ref[k]
        orc.field()
        assert np.array_equal(sim.grid(P.PIC_R_RHO, inst=i), orc.rho)
        tol = 8 * w.nc * EPS64 * np.max(np.abs(orc.phi)) + 1e-300
        assert np.max(np.abs(sim.grid(P.PIC_R_PHI, inst=i) - orc.phi)) <= tol
    sim.close()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_subcycled_ions(prec):
    """Ions pushed every 4 steps over 4 dt (deposited in between), 41 whole steps with
    walls, collisions, source and a sort every 20 steps."""
    wl = pin.bounded_mcc(nc=300, ppc=40, seed=15)
    wl.species[1].nstep = 4
    wl.mcc.n_n *= 5
    flush(f"subcycled ions prec={prec}")
    sim, orc, ost = build_pair(wl, prec)
    sim.step(41, sort_every=20)
    orc.step(41)
    d, rc = sim.diagnostics()
    d = d[0]
    c = orc.counters
    od = orc.diagnostics()
    assert rc == 0 and d.step == 41
    if prec == FP64:
        assert d.particle_steps == c.particle_steps
        assert d.n_cx == c.n_cx and d.n_ionize == c.n_ionize and d.n_source == c.n_source
        for k in range(2):
            g, o = gpu_state(sim, k), oracle_state(orc, k)
            assert np.array_equal(g["id"], o["id"])
            assert np.max(np.abs(g["x"] - o["x"])) <= 1e-7
            assert abs(d.ke[k] / od.ke[k] - 1) <= 1e-9
    else:
        assert abs(d.particle_steps - c.particle_steps) <= 0.001 * c.particle_steps
        for k in range(2):
            assert abs(d.ke[k] / od.ke[k] - 1) <= 5e-3
    sim.close()


def test_more_segments_than_the_lds_tables_fp64():
    """600 small instances (1200 segments): more segments than the movers, the
    sort and the collide kernel stage in LDS (1024), so their global-memory
    paths run.  Every instance against its own oracle: identical ids and
    process counts."""
    wls = pin.batched(n_inst=600, seed=61, nc_min=32, nc_ratio=2.0, ppc_range=(20.0, 40.0))
    for w in wls:
        w.mcc.n_n *= 20  # collisions in every instance
    states = [pin.initial_state(w) for w in wls]
    caps = [pin.capacities(w, s) for w, s in zip(wls, states)]
    flush("600 instances, 1200 segments")
    sim = P.PicSim(wls, states, FP64, capacities=caps, flags=P.PIC_INIT_SORT)
    sim.step(12, sort_every=6)
    d, rc = sim.diagnostics()
    assert rc == 0
    tot = 0
    for i, (w, s) in enumerate(zip(wls, states)):
        orc = oracle.OracleSim(w, s, caps=caps[i], inst=i)
        orc.step(12)
        c = orc.counters
        assert (d[i].n_candidates, d[i].n_elastic, d[i].n_ionize, d[i].n_cx) == \
            (c.n_candidates, c.n_elastic, c.n_ionize, c.n_cx), i
        tot += c.n_elastic
        if i % 37 == 0:
            for k in range(2):
                g = by_id(sim.state(k, inst=i))
                o = oracle_state(orc, k)
                assert np.array_equal(g["id"], o["id"]), (i, k)
                assert np.max(np.abs(g["x"] - o["x"]), initial=0.0) <= 1e-7
    assert tot > 1000
    sim.close()


def test_bounded_8192_cells_full_shape():
    """The bounded magnetised plasma at its full shape (8,192 cells, 200
    particles per cell per species, 3.3e6 particles, B at 45 degrees with
    omega_ce dt = 0.2, pair source, sort every 20 steps).  FP64 form: 25 whole
    steps (one sort) against the oracle, every particle by id.  FP32 form: the
    deposit of the whole uploaded state bit-exact, then one push compared with
    the oracle's push on a sample of 20,000 particles per species."""
    wl = pin.bounded()
    assert wl.nc == 8192 and wl.source and wl.mcc is None
    flush("bounded 8192 cells: FP64, 25 steps")
    sim, orc, ost = build_pair(wl, FP64)
    sim.step(25, sort_every=20)
    orc.step(25)
    d, rc = sim.diagnostics()
    d = d[0]
    od = orc.diagnostics()
    c = orc.counters
    assert rc == 0 and d.status == 0 and d.step == 25
    assert d.n_source == c.n_source and d.next_id == c.next_id and c.n_source > 0
    for k in range(2):
        assert d.n_live[k] == od.n[k]
        assert list(d.absorbed_total[k]) == list(c.absorbed_total[k])
        g, o = gpu_state(sim, k), oracle_state(orc, k)
        assert np.array_equal(g["id"], o["id"])
        assert np.max(np.abs(g["x"] - o["x"])) <= 1e-7
        assert abs(d.ke[k] / od.ke[k] - 1) <= 1e-9
    _check_momentum(d, od, wl, 1e-9)
    sim.close()

    flush("bounded 8192 cells: FP32 deposit and one sampled push")
    st = pin.initial_state(wl)
    st32 = pin.to_fp32_form(st, wl.nc)
    ost = [s.as_f64() for s in st32]
    caps = pin.capacities(wl, st)
    sim = P.PicSim(wl, st32, FP32, capacities=caps, flags=P.PIC_INIT_NO_FIELD)
    sim.deposit()
    S = sim.grid(P.PIC_R_DEPOSIT)
    for k in range(2):
        assert np.array_equal(S[k], oracle.deposit_fixed(ost[k].x, wl.nc))
    sim.close()
    sim = P.PicSim(wl, st32, FP32, capacities=caps)
    sim.push(P.PIC_PUSH_NO_DEPOSIT)
    full = oracle.OracleSim(wl, ost, caps=caps)
    full.deposit()
    full.field()
    rng = np.random.default_rng(2)
    empty = pin.SpeciesState(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0),
                             id=np.zeros(0, np.uint64))
    for k, s in enumerate(wl.species):
        pick = np.sort(rng.choice(ost[k].n, 20000, replace=False))
        sub = pin.SpeciesState(x=ost[k].x[pick], vx=ost[k].vx[pick], vy=ost[k].vy[pick],
                               vz=ost[k].vz[pick], id=ost[k].id[pick])
        o = oracle.OracleSim(wl, [sub if q == k else empty for q in range(2)], caps=[pick.size + 1] * 2)
        for q in range(2):
            o.acc[q][:] = full.acc[q]
        o.push()
        o.walls()
        os_ = oracle_state(o, k)
        g = gpu_state(sim, k)
        gi = np.searchsorted(g["id"], os_["id"])
        ok = gi < g["id"].size
        gi = np.minimum(gi, g["id"].size - 1)
        ok &= g["id"][gi] == os_["id"]
        assert ok.mean() > 0.999
        vth = wl.vth_hat(s)
        assert np.max(np.abs(g["x"][gi[ok]] - os_["x"][ok])) <= 1e-5
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f][gi[ok]] - os_[f][ok]) / np.maximum(np.abs(os_[f][ok]), vth)
            assert np.max(err) <= 1e-5
    sim.close()


@pytest.mark.parametrize("case", ["uploaded", "created"])
def test_ids_at_or_above_2_32(case):
    """Particle ids are two 32-bit words; the movers read only the low words
    while every id of the instance is below 2^32.  Ids of 2^32 and more --
    uploaded ones (2^36 + i), or created ones once next_id passes 2^32 -- make
    them read both words: 12 FP64 steps with collisions, pairs, source and
    sorts give the oracle's counts, ids and positions."""
    wl = pin.bounded_mcc(nc=256, ppc=40, seed=63)
    wl.mcc.n_n *= 20
    st = pin.initial_state(wl)
    n = int(sum(s.n for s in st))
    if case == "uploaded":
        shift = np.uint64(1 << 36)
        st = [pin.SpeciesState(x=s.x, vx=s.vx, vy=s.vy, vz=s.vz, id=s.id + shift) for s in st]
        next_id = n + (1 << 36)
    else:
        next_id = (1 << 32) - 8
    flush(f"ids at or above 2^32: {case}")
    caps = pin.capacities(wl, st)
    sim = P.PicSim(wl, st, FP64, capacities=caps, next_ids=[next_id])
    orc = oracle.OracleSim(wl, st, caps=caps)
    orc.sim.cnt.next_id = next_id
    sim.step(12, sort_every=5)
    orc.step(12)
    d, rc = sim.diagnostics()
    d = d[0]
    c = orc.counters
    assert rc == 0 and d.status == 0
    assert d.next_id == c.next_id and d.next_id > 2 ** 32
    assert d.n_candidates == c.n_candidates and d.n_ionize == c.n_ionize and c.n_ionize > 0
    for k in range(2):
        g, o = gpu_state(sim, k), oracle_state(orc, k)
        assert np.array_equal(g["id"], o["id"])
        assert np.max(np.abs(g["x"] - o["x"])) <= 1e-7
        assert np.any(g["id"] >= np.uint64(2 ** 32))
    sim.close()
