"""Writes precision_subsample_oracle.json: the oracle's moments of the
10,000-cell instance (200 particles per cell per species, seed 5, MCC and
source on) at steps 500, 1000, 1500 and 2000, from the drawn initial state
that the GPU forms also start from.  This is the small instance beside the
1,000,000-cell precision run (the "1% subsample instance"); bench.py
--precision-study compares the GPU forms with these values.

Calls only the oracle (plain FP64 C) and the input generators.  About three
minutes on one core.

    python tests/golden/make_precision_subsample.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import pic_inputs as pin  # noqa: E402

NC, PPC, SEED = 10_000, 200, 5
CHECKPOINTS = (500, 1000, 1500, 2000)
BINS = 64


def moments(o, wl):
    # The oracle solves the field at the start of a step, the GPU at the end:
    # solve it here from the current positions so that the field energy is
    # that of the same positions (the next step solves it again, unchanged).
    o.deposit()
    o.field()
    d = o.diagnostics()
    out = {"step": o.step_index}
    for k in range(len(wl.species)):
        st = o.state(k)
        out[f"N{k}"] = int(d.n[k])
        out[f"KE{k}"] = float(d.ke[k])
        out[f"h{k}"] = np.histogram(st.x, bins=BINS, range=(0, wl.nc))[0].astype(int).tolist()
    out["FE"] = float(d.field_energy)
    return out


def main():
    wl = pin.bounded_mcc(nc=NC, ppc=PPC, seed=SEED)
    st = oracle.init_state(wl)
    n = sum(int(s.id.shape[0]) for s in st)
    caps = [2 * int(s.id.shape[0]) + 1024 for s in st]
    o = oracle.OracleSim(wl, st, caps=caps)
    rows = [moments(o, wl)]
    t0 = time.perf_counter()
    last = 0
    for c in CHECKPOINTS:
        o.step(c - last)
        last = c
        rows.append(moments(o, wl))
        print(f"step {c}: {time.perf_counter() - t0:.0f} s", flush=True)
    out = {"workload": f"bounded_mcc(nc={NC}, ppc={PPC}, seed={SEED}), drawn initial state, {n} particles",
           "bins": BINS, "caps": caps, "moments": rows}
    with open(os.path.join(HERE, "precision_subsample_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
