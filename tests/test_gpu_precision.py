"""FP32 form against FP64 form over 10^4 steps (the moment tolerance of the
FP32/fixed-point form).  The collisional bounded plasma is chaotic on this
time scale, so the comparison is made against the FP64 run's own noise floor:
the same FP64 run with every initial position moved by one ulp (up and down).
Domain-integrated moments and a 64-bin density profile must stay within
max(1e-4, 3 x the noise floor) of the FP64 run."""
import numpy as np
import pytest

import pic_inputs as pin
from gpu_common import FP32, FP64, P, flush

pytestmark = pytest.mark.gpu

STEPS = 10_000


def _moments(sim, wl):
    d, rc = sim.diagnostics()
    assert rc == 0, f"device status {d[0].status:#x}"
    d = d[0]
    m = {}
    for k in range(2):
        st = sim.state(k)
        m[f"N{k}"] = float(d.n_live[k])
        m[f"KE{k}"] = d.ke[k]
        m[f"h{k}"] = np.histogram(st["x"], bins=64, range=(0, wl.nc))[0].astype(np.float64)
    m["E"] = d.ke[0] + d.ke[1] + d.field_energy
    return m


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))))


@pytest.mark.slow
def test_fp32_moments_track_fp64_over_1e4_steps():
    wl = pin.bounded_mcc(nc=10_000, ppc=200, seed=5)
    n = int(round(200 * wl.nc))
    caps = [4 * n + 1024] * 2  # ionisation grows the plasma by ~80% over 10^4 steps
    flush("precision: FP64 reference")
    ref = P.PicSim(wl, None, FP64, capacities=caps, flags=P.PIC_INIT_DEVICE)
    st0 = [ref.state(k) for k in range(2)]
    ref.step_graph(STEPS, 20)
    m64 = _moments(ref, wl)
    ref.close()
    flush("precision: FP32 form")
    f32 = P.PicSim(wl, None, FP32, capacities=caps, flags=P.PIC_INIT_DEVICE)
    f32.step_graph(STEPS, 20)
    m32 = _moments(f32, wl)
    f32.close()
    floors = []
    for direction in (np.inf, -np.inf):
        flush(f"precision: FP64 with positions moved one ulp towards {direction}")
        pert = []
        for k in range(2):
            x = np.nextafter(st0[k]["x"], direction)
            x = np.where((x >= wl.nc) | (x < 0), st0[k]["x"], x)
            pert.append(pin.SpeciesState(x=x, vx=st0[k]["vx"], vy=st0[k]["vy"], vz=st0[k]["vz"],
                                         id=st0[k]["id"]))
        sim = P.PicSim(wl, pert, FP64, capacities=caps, next_ids=[2 * n])
        sim.step_graph(STEPS, 20)
        floors.append(_moments(sim, wl))
        sim.close()
    for key in ("N0", "N1", "KE0", "KE1", "E", "h0", "h1"):
        floor = max(_rel(f[key], m64[key]) for f in floors)
        err = _rel(m32[key], m64[key])
        flush(f"{key}: fp32-fp64 {err:.3e}, fp64 noise floor {floor:.3e}")
        assert err <= max(1e-4, 3.0 * floor), key


def test_fp64_form_tracks_the_oracle_over_2000_steps():
    """The 10,000-cell precision instance (4e6 particles, MCC and source on),
    drawn on the device, 2,000 steps of the FP64 form against the oracle's
    moments at steps 500..2000 (tests/golden/precision_subsample_oracle.json,
    written by the oracle alone from the same draw).  The two differ only in
    the rounding of the field solve, which over 2,000 steps moves no particle
    across a 64-bin boundary and changes no collision or wall outcome: counts
    and density profiles equal, kinetic energies to summation order, the
    field energy to the solve's rounding."""
    import json
    import os
    gold_path = os.path.join(os.path.dirname(__file__), "golden", "precision_subsample_oracle.json")
    with open(gold_path) as f:
        gold = json.load(f)
    wl = pin.bounded_mcc(nc=10_000, ppc=200, seed=5)
    flush("precision: FP64 form against the stored oracle moments, 2,000 steps")
    sim = P.PicSim(wl, None, FP64, capacities=gold["caps"], flags=P.PIC_INIT_DEVICE)
    last = 0
    for g in gold["moments"][1:]:
        sim.step_graph(g["step"] - last, 20)
        last = g["step"]
        d, rc = sim.diagnostics()
        assert rc == 0 and d[0].step == g["step"]
        for k in range(2):
            assert int(d[0].n_live[k]) == g[f"N{k}"], (g["step"], k)
            h = np.histogram(sim.state(k)["x"], bins=gold["bins"], range=(0, wl.nc))[0]
            assert np.array_equal(h, np.asarray(g[f"h{k}"])), (g["step"], k)
            assert abs(d[0].ke[k] / g[f"KE{k}"] - 1) <= 1e-12, (g["step"], k)
        assert abs(d[0].field_energy / g["FE"] - 1) <= 1e-6, g["step"]
    sim.close()
