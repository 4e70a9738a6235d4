"""Shared set-up of the GPU parity tests: the same seeded state goes to the
HIP path (through the C ABI) and to the oracle; in the FP32 form the oracle
receives the state exactly as rounded for FP32 storage."""
from __future__ import annotations

import numpy as np

import oracle
import pic_inputs as pin
from paper_2404_10270_amd import pic as P

FP32, FP64 = P.PIC_FP32, P.PIC_FP64


def build_pair(wl, precision, caps=None, flags=0, state=None):
    """(PicSim, OracleSim, oracle-side initial state) for one workload."""
    st64 = state if state is not None else pin.initial_state(wl)
    if caps is None:
        caps = pin.capacities(wl, st64)
    if precision == FP32:
        st32 = pin.to_fp32_form(st64, wl.nc)
        dev_state = st32
        orc_state = [s.as_f64() for s in st32]
    else:
        dev_state = st64
        orc_state = st64
    sim = P.PicSim(wl, dev_state, precision, capacities=caps, flags=flags)
    orc = oracle.OracleSim(wl, orc_state, caps=caps)
    return sim, orc, orc_state


def by_id(d):
    """Sort a state dict (numpy arrays) by particle id."""
    o = np.argsort(d["id"], kind="stable")
    return {k: (v[o] if isinstance(v, np.ndarray) and v.shape == d["id"].shape else v)
            for k, v in d.items()}


def oracle_state(orc, k):
    s = orc.state(k)
    return by_id({"x": s.x, "vx": s.vx, "vy": s.vy, "vz": s.vz, "id": s.id})


def gpu_state(sim, k):
    return by_id(sim.state(k))


def flush(msg):
    print(msg, flush=True)
