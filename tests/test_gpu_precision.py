"""FP32 form against FP64 form over 10^4 steps (the moment tolerance of the
FP32/fixed-point form), by the precision protocol fixed before it was
measured: per moment the bound is max(1e-4, spread of an FP64 ensemble), the
ensemble being the FP64 run R and 16 FP64 runs whose drawn start has every
position moved by one ulp (signs from a device generator seeded 1000 + i),
with no free factor.  Moments: N and kinetic energy per species, field
energy, total energy, 64-bin density profile per species.  The protocol is
bench.precision_protocol; the same code writes the precision study's JSON."""
import numpy as np
import pytest

import pic_inputs as pin
from gpu_common import FP64, P, flush

pytestmark = pytest.mark.gpu

STEPS = 10_000


@pytest.mark.slow
def test_fp32_moments_within_the_fp64_ensemble_over_1e4_steps():
    import torch

    import bench
    wl = pin.bounded_mcc(nc=10_000, ppc=200, seed=5)
    n = int(round(200 * wl.nc))
    caps = [4 * n + 1024] * 2  # ionisation grows the plasma by ~80% over 10^4 steps
    flush("precision protocol: 10,000 cells, 4e6 particles, 10^4 steps, 17-run FP64 ensemble")
    res = bench.precision_protocol(torch, wl, caps, STEPS, 16, P.PIC_INIT_DEVICE)
    assert res["ensemble"] == 17 and res["steps"] == STEPS
    for key, m in res["moments"].items():
        flush(f"{key}: FP32 {m['fp32_dev']:.3e}, FP64 spread {m['fp64_spread']:.3e}, "
              f"bound {m['bound']:.3e} ({m['binds']})")
        assert m["bound"] == max(1e-4, m["fp64_spread"])
        assert m["fp32_dev"] <= m["bound"], key
    # the perturbed runs really differ from R (the spread is not a rounding artefact)
    assert res["moments"]["N0"]["fp64_spread"] > 0


def test_one_ulp_perturbation_moves_every_position_by_one_ulp():
    """The ensemble's perturbation: every drawn position moves to a neighbouring
    double (up or down, about half each way), none leaves [0, nc), and the
    deposit and field are formed from the moved positions as pic_init forms them."""
    import torch

    import bench
    wl = pin.bounded_mcc(nc=300, ppc=50, seed=5)
    ref = P.PicSim(wl, None, FP64, flags=P.PIC_INIT_DEVICE)
    x0 = [ref.state(k)["x"] for k in range(2)]
    ref.close()
    sim = P.PicSim(wl, None, FP64, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_NO_FIELD)
    bench.perturb_one_ulp(torch, sim, wl.nc, 1001)
    rho = sim.grid(P.PIC_R_RHO)
    for k in range(2):
        x = sim.state(k)["x"]
        up = x == np.nextafter(x0[k], np.inf)
        dn = x == np.nextafter(x0[k], -np.inf)
        assert np.all(up | dn | (x == x0[k])) and np.all((x >= 0) & (x < wl.nc))
        assert 0.45 < up.mean() < 0.55 and 0.45 < dn.mean() < 0.55
    # the same positions uploaded through pic_init give the same charge density
    st = [pin.SpeciesState(x=sim.state(k)["x"], vx=sim.state(k)["vx"], vy=sim.state(k)["vy"],
                           vz=sim.state(k)["vz"], id=sim.state(k)["id"]) for k in range(2)]
    sim.close()
    up_sim = P.PicSim(wl, st, FP64)
    assert np.array_equal(up_sim.grid(P.PIC_R_RHO), rho)
    up_sim.close()


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
