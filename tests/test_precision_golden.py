"""The stored oracle moments of the 10,000-cell precision instance
(tests/golden/precision_subsample_oracle.json, written by
tests/golden/make_precision_subsample.py from the oracle alone): the file is
complete and self-consistent.  The GPU comparison is in test_gpu_precision.py."""
import json
import os

import numpy as np

import oracle
import pic_inputs as pin

GOLD = os.path.join(os.path.dirname(__file__), "golden", "precision_subsample_oracle.json")


def test_golden_moments_are_complete_and_consistent():
    with open(GOLD) as f:
        g = json.load(f)
    rows = g["moments"]
    assert [r["step"] for r in rows] == [0, 500, 1000, 1500, 2000]
    for r in rows:
        for k in range(2):
            h = np.asarray(r[f"h{k}"])
            assert h.shape == (g["bins"],) and h.sum() == r[f"N{k}"]
            assert r[f"KE{k}"] > 0.0
        assert r["FE"] >= 0.0
    # the drawn start: 200 particles per cell per species on 10,000 cells
    assert rows[0]["N0"] == rows[0]["N1"] == 2_000_000


def test_golden_start_is_the_oracle_draw():
    """Step 0 of the file is the oracle's drawn initial state (density profile
    and kinetic energy recomputed here from a fresh draw)."""
    with open(GOLD) as f:
        g = json.load(f)
    wl = pin.bounded_mcc(nc=10_000, ppc=200, seed=5)
    st = oracle.init_state(wl)
    r0 = g["moments"][0]
    for k in range(2):
        h = np.histogram(st[k].x, bins=g["bins"], range=(0, wl.nc))[0]
        assert np.array_equal(h, np.asarray(r0[f"h{k}"]))
