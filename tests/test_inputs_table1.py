"""The Table 1 workload builder against the values the paper prints for its
test case (Sec. 3.4, Table 1), stored in tests/golden/table1_case.txt."""
import math
import os

import pic_inputs as pin

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_case.txt")


def load_golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_table1_workload_matches_the_printed_case():
    g = load_golden()
    wl = pin.table1()
    assert wl.nc == int(g["cells"])
    assert math.isclose(wl.nc * wl.dx, g["system_size_m"], rel_tol=1e-12)
    assert math.isclose(wl.dx, g["cell_size_m"], rel_tol=1e-12)
    assert math.isclose(wl.dt, g["dt_s"], rel_tol=1e-12)
    assert wl.n_steps == int(g["steps"])
    assert math.isclose(wl.n_steps * wl.dt, g["simulated_time_s"], rel_tol=1e-12)
    assert wl.bc == pin.BC_PERIODIC
    assert wl.field_off and wl.B0 == 0.0 and wl.smooth_passes == 0
    assert len(wl.species) == int(g["species"])
    for s in wl.species:
        assert s.ppc == g["ppc_per_species"]
        # macro weight x particles per cell / cell size = physical density
        assert math.isclose(s.w * s.ppc / wl.dx, g["density_m3"], rel_tol=1e-12)
    # electrons and deuterium ions, opposite unit charges, and deuterium atoms
    e, i, n = wl.species
    assert e.kind == pin.KIND_ELECTRON and i.kind == pin.KIND_ION
    assert n.kind == pin.KIND_NEUTRAL and n.q == 0.0
    assert e.q == -i.q
    assert 3600 < i.m / e.m < 3700
    assert math.isclose(n.m, i.m + e.m, rel_tol=1e-12)
    for s in (e, i):
        assert math.isclose(s.T / pin.EV, g["T_charged_eV"], rel_tol=1e-12)
    assert math.isclose(n.T / pin.EV, g["T_neutral_eV"], rel_tol=1e-12)
    # electron-neutral processes only
    assert wl.mcc.sig_cx == 0.0 and wl.mcc.sig_el > 0 and wl.mcc.sig_ex > 0 and wl.mcc.sig_iz > 0


def test_table1_particle_count():
    g = load_golden()
    wl = pin.table1()
    assert wl.n_particles == int(g["cells"] * g["ppc_per_species"] * g["species"])
    assert wl.n_particles == int(g["particles_total"])
