"""pic_init_static, the entry point for callers that cannot allocate device
memory, against pic_init: the same initial state and steps give the same
particles (by id, bit for bit) and the same diagnostics.  Two static contexts
in a row, the second on a smaller workload (the static array then holds the
first one's leftovers); a second live static context on the device is
refused until the first is destroyed."""
import numpy as np
import pytest

import pic_inputs as pin
from gpu_common import FP32, FP64, P, by_id, flush

pytestmark = pytest.mark.gpu

COUNTS = ("step", "next_id", "status", "n_candidates", "n_elastic", "n_ionize", "n_cx",
          "n_over_cap", "n_source", "particle_steps")


def _run(wl, prec, static_work, flags, steps, sort_every, state, caps):
    sim = P.PicSim(wl, state, prec, capacities=caps, flags=flags, static_work=static_work)
    try:
        sim.step(steps, sort_every)
        d, rc = sim.diagnostics()
        assert rc == 0, f"device status {d[0].status:#x}"
        parts = [by_id(sim.state(k)) for k in range(sim.nsp)]
    finally:
        sim.close()
    return d[0], parts


def _compare(a, b, nsp):
    da, pa = a
    db, pb = b
    for f in COUNTS:
        assert getattr(da, f) == getattr(db, f), f
    for k in range(nsp):
        assert da.n_live[k] == db.n_live[k] and da.n_slots_used[k] == db.n_slots_used[k], k
        assert da.created_total[k] == db.created_total[k], k
        assert list(da.absorbed_total[k]) == list(db.absorbed_total[k]), k
        assert da.ke[k] == pytest.approx(db.ke[k], rel=1e-13, abs=0.0), k
        for c in range(3):
            assert da.mom[k][c] == pytest.approx(db.mom[k][c], rel=1e-12, abs=1e-300), (k, c)
        for f in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(pa[k][f], pb[k][f]), (k, f)
    assert da.field_energy == pytest.approx(db.field_energy, rel=1e-13, abs=0.0)


@pytest.mark.parametrize("case", [
    # (workload, form, init flags, steps, sort cadence): the second is smaller
    ("bounded_mcc nc=512 ppc=40, FP64, uploaded and sorted", 512, 40, FP64,
     P.PIC_INIT_SORT, 12, 5),
    ("bounded_mcc nc=256 ppc=20, FP32, drawn on the device", 256, 20, FP32,
     P.PIC_INIT_DEVICE, 9, 4),
])
def test_static_workspace_matches_pic_init(case):
    name, nc, ppc, prec, flags, steps, sort_every = case
    flush(f"no-alloc entry point: {name}")
    wl = pin.bounded_mcc(nc=nc, ppc=ppc, seed=41)
    wl.mcc.n_n *= 10  # more collisions and ionisation pairs per step
    if flags & P.PIC_INIT_DEVICE:
        state = None
        caps = [int(2 * ppc * nc) + 1024] * 2
    else:
        st64 = pin.initial_state(wl)
        state = pin.to_fp32_form(st64, wl.nc) if prec == FP32 else st64
        caps = pin.capacities(wl, st64)
    ref = _run(wl, prec, False, flags, steps, sort_every, state, caps)
    got = _run(wl, prec, True, flags, steps, sort_every, state, caps)
    _compare(got, ref, 2)


def test_static_workspace_is_held_by_one_context():
    wl = pin.bounded_mcc(nc=128, ppc=10, seed=43)
    st = pin.initial_state(wl)
    flush("no-alloc entry point: one live context per device")
    a = P.PicSim(wl, st, FP64, static_work=True)
    try:
        with pytest.raises(P.PicError) as e:
            P.PicSim(wl, st, FP64, static_work=True)
        assert e.value.code == P.PIC_E_BUSY
    finally:
        a.close()
    b = P.PicSim(wl, st, FP64, static_work=True)  # released by pic_destroy
    b.close()
