#!/usr/bin/env python3
"""Throughput of the 1D3V PIC-MCC hot path on one MI355X.

Workload: the collisional bounded plasma -- 100,000 cells between two
grounded absorbing walls, electrons and ions (m_i/m_e = 1836, 20 eV),
100 particles per cell per species (2e7 particles), B at 45 degrees with
omega_ce dt = 0.2, null-collision MCC against a neutral gas (elastic,
charge exchange, ionisation), pair source, cell sort every 20 steps.  FP32
push with 64-bit fixed-point deposition (the FP64 form is timed beside it).
Inputs are seeded and synthetic (pic_inputs) and resident in HBM before the
timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` = particles pushed per second over the K timed
steps (every step runs push+deposit+candidate test, collisions, pairs and
source, field solve, and a sort every 20 steps).  `roofline` is for the
dominant kernel (the fused mover), timed with HIP events on its stream;
`windows` gives the median, least and largest rate of five further one-period
windows.  Beside it: the FP64 form, the 4e8-particle instance on 1,000,000
cells in both forms, the two small configurations (Langmuir, 8,192-cell
bounded plasma), 256 batched instances, the paper's own Table 1 test case
(electrons, D+ ions and kinetic D atoms, no field solve), and the oracle on
the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle and push: read cell, f, vx, vy, vz (4 B each)
# and the id's low word (4 B: every id of the workloads is below 2^32); write
# cell, f, vx, vy, vz
PUSH_BYTES_FP32 = 5 * 4 + 4 + 5 * 4
# FP64 form: read x, vx, vy, vz (8 B each) and the id's low word; write x, vx, vy, vz
PUSH_BYTES_FP64 = 4 * 8 + 4 + 4 * 8
SORT_EVERY = 20
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "push_f32_bounded_mcc_traffic.json")
PUSH_SOURCES = ["paper_2404_10270_amd/csrc/push.hip", "paper_2404_10270_amd/csrc/device_common.h",
                "paper_2404_10270_amd/csrc/pic_internal.h", "paper_2404_10270_amd/csrc/mover_common.h",
                "paper_2404_10270_amd/csrc/collide_common.h", "paper_2404_10270_amd/csrc/tile_queue.h"]
# the mover bench.py times for the roofline: pic_push's launch (push, deposit
# and candidate list; the step's launch also collides the block's own
# candidates)
MOVER_KERNEL = "push_f32_kernel<true, true, 4, false>"
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written per launch


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload(args):
    import pic_inputs as pin
    return pin.bounded_mcc(nc=args.nc, ppc=args.ppc, seed=3, sort_every=SORT_EVERY,
                           cap_factor=1.25)


def make_sim(wl, st64, precision):
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P
    caps = pin.capacities(wl, st64)
    state = pin.to_fp32_form(st64, wl.nc) if precision == P.PIC_FP32 else st64
    return P.PicSim(wl, state, precision, capacities=caps, flags=P.PIC_INIT_SORT)


def mover_shapes(sim):
    """Candidate launch shapes of the mover: 4 chunks per wave in one pass or 2
    in two passes, on the default grid or on the largest one."""
    nmax = int(sim.sizes.mover_blocks_max)
    shapes = [(4, 0), (2, 0)]
    if nmax > int(sim.sizes.mover_blocks):
        shapes += [(4, nmax), (2, nmax)]
    return shapes


def tune_mover(sim, trial_steps=80):
    """Autotune the mover's launch shape at the workload's sort cadence."""
    movers = mover_shapes(sim)
    best, _, rates, _ = sim.autotune(movers, (SORT_EVERY,), trial_steps)
    return {"chunks": best[0], "blocks": best[1] or int(sim.sizes.mover_blocks),
            "trials": {f"{m[0]}x{m[1] or int(sim.sizes.mover_blocks)}": round(r, 1)
                       for m, r in zip(movers, rates)}}


def tuned_sim(torch, make):
    """The mover's launch shape chosen on a throwaway copy of the workload
    (make() builds one), then a fresh copy set to that shape: the trials run
    hundreds of steps, over which ionisation grows the plasma, so the timed
    run starts from the workload's own initial state."""
    sim = make()
    shape = tune_mover(sim)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    sim = make()
    sim.set_mover(shape["chunks"], shape["blocks"])
    return sim, shape


def run_form(torch, sim, steps, warmup, graph=False):
    """Time `steps` whole steps after `warmup`; returns (p-steps/s, ms/step, p-steps).
    With `graph` the steps are replayed from a captured HIP graph (pic_step_graph)."""
    step = sim.step_graph if graph else sim.step
    step(warmup, SORT_EVERY)
    if graph:
        sim.step_graph(0, SORT_EVERY)  # the period graph for this phase, captured untimed
    d0, _ = sim.diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(steps, SORT_EVERY)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1, rc = sim.diagnostics()
    if rc != 0:
        raise RuntimeError(f"device status {d1[0].status:#x} during the timed region")
    ps = int(d1[0].particle_steps - d0[0].particle_steps)
    dt = t1 - t0
    return ps / dt, 1e3 * dt / steps, ps


def time_windows(torch, sim, n_windows=5, steps=SORT_EVERY, sort_every=SORT_EVERY):
    """Rate of `n_windows` further windows of `steps` whole steps each (one
    sort period), replayed from the HIP graph and timed with HIP events on the
    context's stream: median, least and largest p-steps/s."""
    import statistics
    rates = []
    for _ in range(n_windows):
        d0, _ = sim.diagnostics()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step_graph(steps, sort_every)
        e1.record(sim.stream)
        d1, rc = sim.diagnostics()
        if rc != 0:
            raise RuntimeError(f"device status {d1[0].status:#x} in a timed window")
        ps = sum(int(d1[i].particle_steps - d0[i].particle_steps) for i in range(len(d1)))
        rates.append(ps / (e0.elapsed_time(e1) * 1e-3))
    return {"windows": n_windows, "steps_each": steps, "median": statistics.median(rates),
            "min": min(rates), "max": max(rates)}


def time_push(torch, sim, n_steps):
    """Average duration of the mover launch pic_push makes (push, fused deposit
    and candidate list), HIP events on its stream, between whole steps."""
    from paper_2404_10270_amd import pic as P
    d0, _ = sim.diagnostics()
    evs = []
    step = int(d0[0].step)
    for _ in range(n_steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.push()
        e1.record(sim.stream)
        sim.mcc_collide()
        sim.field_solve()
        step += 1
        if step % SORT_EVERY == 0:
            sim.sort()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    d1, _ = sim.diagnostics()
    ms = [a.elapsed_time(b) for a, b in evs]
    per_launch = (d1[0].particle_steps - d0[0].particle_steps) / n_steps
    return sum(ms) / len(ms), per_launch


def traffic_from_profile():
    """HBM bytes per mover launch from the committed rocprofv3 counter summary,
    or None when the mover's source changed since the counters were taken."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash(PUSH_SOURCES):
        return None
    return t.get("bytes_per_launch")


def copy_calibration():
    """A plain elementwise copy of known size (torch.neg, 1 GiB in, 1 GiB out),
    launched 5 times, for scaling the HBM byte counters."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES,
                      "launches": 5}), flush=True)


def copy_rate(torch):
    """HBM bandwidth a plain copy reaches (torch.neg, 1 GiB in and 1 GiB out),
    timed with HIP events over 5 launches after one warm-up: what a streaming
    kernel attains on this GPU, beside the 8 TB/s peak."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(5):
        torch.neg(src, out=dst)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del src, dst
    torch.cuda.empty_cache()
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def _pmc_rows(d, kernel_sub, counter):
    """Per-dispatch values of `counter` for kernels whose name contains
    `kernel_sub`, from a rocprofv3 --pmc CSV directory."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    vals = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if kernel_sub in r["Kernel_Name"] and r["Counter_Name"] == counter:
                    key = (fn, r["Dispatch_Id"])
                    vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise ValueError(f"no {counter} rows for '{kernel_sub}' under {d}")
    return list(vals.values())


def pmc_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, out):
    """HBM bytes per mover launch: FETCH_SIZE and WRITE_SIZE of the mover,
    each scaled by bytes / counter value of the calibration copy."""
    import statistics
    mover = MOVER_KERNEL
    cf = statistics.mean(_pmc_rows(cfetch_dir, "neg_kernel", "FETCH_SIZE"))
    cw = statistics.mean(_pmc_rows(cwrite_dir, "neg_kernel", "WRITE_SIZE"))
    f_fetch, f_write = COPY_BYTES / cf, COPY_BYTES / cw
    mf = _pmc_rows(fetch_dir, mover, "FETCH_SIZE")
    mw = _pmc_rows(write_dir, mover, "WRITE_SIZE")
    fetch_b = statistics.mean(mf) * f_fetch
    write_b = statistics.mean(mw) * f_write
    res = {"kernel": mover, "source_hash": source_hash(PUSH_SOURCES),
           "bytes_per_launch": round(fetch_b + write_b),
           "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
           "launches": [len(mf), len(mw)],
           "copy_factor": {"FETCH_SIZE": f_fetch, "WRITE_SIZE": f_write},
           "copy_counter_per_launch": {"FETCH_SIZE": cf, "WRITE_SIZE": cw}}
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print(json.dumps(res))


def batched(torch, args):
    """256 independent bounded MCC instances of mixed shape (256 to 16,384 cells,
    25 to 200 particles per cell per species, B at 0 to 85 degrees, omega_pe dt
    0.05 to 0.2) in one context, FP32 form, drawn on the device; the sort
    cadence is chosen by pic_autotune_sort, then steps replay from a HIP graph."""
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P
    wls = pin.batched(n_inst=args.batched_instances, seed=4)
    n = sum(w.n_particles for w in wls)
    log(f"batched: {len(wls)} instances, {n} particles, drawn on the device")
    def make():
        return P.PicSim(wls, [None] * len(wls), P.PIC_FP32, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_SORT)
    # shape and cadence chosen on a throwaway copy (see tuned_sim)
    sim = make()
    cands = (5, 10, 20, 40, 80)
    movers = mover_shapes(sim)
    mover, best, mrates, rates = sim.autotune(movers, cands, 80)
    log(f"batched: autotuned mover {mover} ({', '.join(f'{m}: {r:.3e}' for m, r in zip(movers, mrates))}), "
        f"sort cadence {best} ({', '.join(f'{c}: {r:.3e}' for c, r in zip(cands, rates))})")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    sim = make()
    sim.set_mover(mover[0], mover[1])
    # one untimed sort period (the graph is captured in it), then whole periods
    # (each with its sort), at least --batched-steps steps
    period = best if best > 0 else 20
    steps = period * max(1, -(-args.batched_steps // period))
    sim.step_graph(period, best)
    d0, _ = sim.diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step_graph(steps, best)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d1, rc = sim.diagnostics()
    if rc != 0:
        raise RuntimeError(f"device status during the batched run: {rc}")
    ps = sum(int(d1[i].particle_steps - d0[i].particle_steps) for i in range(len(wls)))
    sim.close()
    out = {"value": ps / dt, "unit": "particle-steps/s", "instances": len(wls), "particles": n,
           "cells": sum(w.nc for w in wls), "steps": steps,
           "ms_per_step": round(1e3 * dt / steps, 4), "sort_every": best,
           "mover": {"chunks": mover[0], "blocks": mover[1] or int(sim.sizes.mover_blocks)},
           "autotune": {"mover": {f"{m[0]}x{m[1] or int(sim.sizes.mover_blocks)}": round(r, 1)
                                  for m, r in zip(movers, mrates)},
                        "sort_every": {str(c): round(r, 1) for c, r in zip(cands, rates)}}}
    log(f"batched: {out['value']:.4e} p-steps/s, {out['ms_per_step']} ms/step")
    return out


def table1_run(torch, args):
    """The paper's Table 1 test case at full size (Sec. 3.4): electrons, D+ ions
    and kinetic D atoms, 100,000 cells x 100 particles per cell per species (3e7
    particles), 1 m, dt = 4e-14 s, periodic, no field solve; elastic, excitation
    and ionisation against the atoms (stand-in cross sections); FP32 form, drawn
    on the device and sorted, steps from a HIP graph with a sort every 20 steps.
    The mover moves 44 B per electron (its id's low word is read for the
    collision test) and 40 B per ion or atom (no process, no id read)."""
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P
    wl = pin.table1()
    n = wl.n_particles
    log(f"table1: {n} particles on {wl.nc} cells, drawn on the device")
    sim = P.PicSim(wl, None, P.PIC_FP32, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_SORT)
    rate, ms_step, _ = run_form(torch, sim, args.table1_steps, args.warmup, graph=True)
    d0, _ = sim.diagnostics()
    push_ms, per_launch = time_push(torch, sim, args.push_steps)
    d1, rc = sim.diagnostics()
    if rc != 0:
        raise RuntimeError(f"device status during the table1 run: {rc}")
    live = [int(d1[0].n_live[k]) for k in range(3)]
    bytes_launch = PUSH_BYTES_FP32 * live[0] + (PUSH_BYTES_FP32 - 4) * (live[1] + live[2])
    gbs = bytes_launch / (push_ms * 1e-3) / 1e9
    sim.close()
    out = {"value": rate, "unit": "particle-steps/s", "particles": n, "cells": wl.nc,
           "steps": args.table1_steps, "ms_per_step": round(ms_step, 4), "sort_every": SORT_EVERY,
           "field_solve": "off", "mover_us": round(push_ms * 1e3, 2),
           "mover_GBps": round(gbs, 1), "mover_frac": round(gbs / HBM_PEAK_GBS, 4),
           "ionisations": int(d1[0].n_ionize), "atoms_consumed": int(d1[0].n_consumed)}
    log(f"table1: {rate:.4e} p-steps/s, {ms_step:.4f} ms/step, mover {push_ms * 1e3:.1f} us "
        f"({gbs:.0f} GB/s)")
    return out


PRECISION_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                                "precision_subsample_oracle.json")


def _gpu_moments(torch, sim, nc, bins):
    """N, kinetic energy and a `bins`-bin density histogram per species, and
    the field energy, of instance 0 (histograms from the device arrays)."""
    from paper_2404_10270_amd import pic as P
    d, rc = sim.diagnostics()
    if rc != 0:
        raise RuntimeError(f"device status {d[0].status:#x}")
    d = d[0]
    cur = d.cur_set
    out = {"step": int(d.step)}
    for k in range(sim.nsp):
        b = sim.seg_base[k]
        m = int(d.n_slots_used[k])
        if sim.precision == P.PIC_FP32:
            c = sim.cell[cur][b:b + m]
            live = c >= 0
            x = c[live].double() + sim.x[cur][b:b + m][live].double()
        else:
            x = sim.x[cur][b:b + m]
            x = x[x >= 0]
        idx = torch.clamp(torch.floor(x * (bins / nc)).long(), 0, bins - 1)
        out[f"N{k}"] = int(d.n_live[k])
        out[f"KE{k}"] = float(d.ke[k])
        out[f"h{k}"] = torch.bincount(idx, minlength=bins).cpu().tolist()
    out["FE"] = float(d.field_energy)
    return out


def _rel_diff(a, b):
    """Largest relative difference of moments a against b (histograms: over bins)."""
    import numpy as np
    r = {}
    for key in b:
        if key == "step":
            continue
        x, y = np.asarray(a[key], np.float64), np.asarray(b[key], np.float64)
        r[key] = float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1e-300)))
    return r


PRECISION_BINS = 64


def perturb_one_ulp(torch, sim, nc, seed):
    """Move every particle position of an FP64-form context (current buffer
    set) by one ulp, up or down by a fair sign per particle drawn from a
    device torch.Generator seeded `seed` (species in order); a position that
    would leave [0, nc) keeps its value.  Then deposit and solve the field, as
    pic_init does after its draw (the context is made with PIC_INIT_NO_FIELD)."""
    from paper_2404_10270_amd import pic as P
    if sim.precision != P.PIC_FP64:
        raise ValueError("the one-ulp ensemble perturbs the FP64 form")
    d, _ = sim.diagnostics()
    cur = d[0].cur_set
    dev = sim.x[cur].device
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    inf = torch.tensor(float("inf"), dtype=torch.float64, device=dev)
    for k in range(sim.nsp):
        b = sim.seg_base[k]
        m = int(d[0].n_slots_used[k])
        x = sim.x[cur][b:b + m]
        up = torch.randint(0, 2, (m,), generator=g, device=dev, dtype=torch.int8) == 1
        y = torch.where(up, torch.nextafter(x, inf), torch.nextafter(x, -inf))
        x.copy_(torch.where((y < 0) | (y >= nc), x, y))
    torch.cuda.synchronize()
    sim.deposit()
    sim.field_solve()


def _protocol_moments(torch, sim, nc):
    m = _gpu_moments(torch, sim, nc, PRECISION_BINS)
    m["E"] = sum(m[f"KE{k}"] for k in range(sim.nsp)) + m["FE"]
    return m


def precision_protocol(torch, wl, caps, steps, K, flags, label=""):
    """The precision protocol (fixed before it was measured): the FP32/fixed-point
    form's moments after `steps` steps against the FP64 form R, with the bound
    per moment max(1e-4, spread of an FP64 ensemble).  The ensemble is R and K
    FP64 runs whose drawn start has every position moved by one ulp (run i:
    signs from a device generator seeded 1000 + i).  Moments: live particles
    N and kinetic energy KE per species, field energy FE, total energy E, and
    a 64-bin density profile h per species.  spread = (largest - smallest over
    the K + 1 runs) / |R| (a profile: per bin, then the largest bin); the FP32
    deviation e = |FP32 - R| / |R| (a profile: the largest bin) passes iff
    e <= max(1e-4, spread).  All runs are drawn on the device (`flags`)."""
    import numpy as np
    from paper_2404_10270_amd import pic as P

    def run(prec, seed=None):
        f = flags | (P.PIC_INIT_NO_FIELD if seed is not None else 0)
        sim = P.PicSim(wl, None, prec, capacities=caps, flags=f)
        try:
            if seed is not None:
                perturb_one_ulp(torch, sim, wl.nc, seed)
            t0 = time.perf_counter()
            sim.step_graph(steps, SORT_EVERY)
            m = _protocol_moments(torch, sim, wl.nc)
        finally:
            sim.close()
            torch.cuda.empty_cache()
        name = "FP32" if prec == P.PIC_FP32 else ("FP64" if seed is None else f"FP64 ulp {seed}")
        log(f"precision{label}: {name} run, {steps} steps in {time.perf_counter() - t0:.1f} s")
        return m

    ens = [run(P.PIC_FP64)]
    ens += [run(P.PIC_FP64, 1000 + i) for i in range(1, K + 1)]
    f32 = run(P.PIC_FP32)
    ref = ens[0]
    keys = [f"N{k}" for k in range(len(wl.species))] + [f"KE{k}" for k in range(len(wl.species))]
    keys += ["FE", "E"] + [f"h{k}" for k in range(len(wl.species))]
    out = {}
    for key in keys:
        vals = np.array([np.asarray(m[key], np.float64) for m in ens])
        den = np.maximum(np.abs(vals[0]), 1e-300)
        spread = float(np.max((vals.max(axis=0) - vals.min(axis=0)) / den))
        dev = float(np.max(np.abs(np.asarray(f32[key], np.float64) - vals[0]) / den))
        bound = max(1e-4, spread)
        out[key] = {"fp32_dev": dev, "fp64_spread": spread, "bound": bound,
                    "binds": "spread" if spread > 1e-4 else "1e-4", "pass": bool(dev <= bound)}
        log(f"precision{label}: {key} FP32 {dev:.3e}, FP64 spread {spread:.3e}, "
            f"{'pass' if dev <= bound else 'FAIL'}")
    return {"steps": steps, "ensemble": K + 1, "moments": out,
            "fp64_R": {k: ref[k] for k in keys if not k.startswith("h")},
            "fp32": {k: f32[k] for k in keys if not k.startswith("h")}}


def precision_study(torch, args):
    """The precision study (FP32/fixed-point form against the FP64 form).
    1. The precision protocol on the 10,000-cell instance (200 particles per
       cell per species, 4e6 particles, MCC and source) over 10^4 steps, with a
       16-run FP64 ensemble.
    2. The same instance (the 1% subsample of the precision configuration)
       over 2,000 steps as both GPU forms, compared with the oracle's moments
       at steps 500..2000 (tests/golden/precision_subsample_oracle.json,
       written by the oracle alone).
    3. The precision protocol on the 1,000,000-cell instance (4e8 particles)
       over 2,000 steps, with an 8-run FP64 ensemble.
    All drawn on the device."""
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P
    bins = PRECISION_BINS
    out = {"protocol": "bound per moment max(1e-4, FP64 one-ulp ensemble spread); FP32 passes "
                       "iff |FP32 - FP64| / |FP64| <= bound"}
    wl = pin.bounded_mcc(nc=10_000, ppc=200, seed=5)
    n = int(round(200 * wl.nc))
    if not args.precision_skip_small:
        caps = [4 * n + 1024] * 2  # ionisation grows the plasma by ~80% over 10^4 steps
        out["instance_10k_cells"] = precision_protocol(torch, wl, caps, 10_000, 16, P.PIC_INIT_DEVICE,
                                                       " (10,000 cells)")
    # ---- the 1% subsample against the oracle's moments
    with open(PRECISION_GOLDEN) as f:
        gold = json.load(f)
    checks = [r["step"] for r in gold["moments"][1:]]
    runs = {}
    for name, prec in (("fp64", P.PIC_FP64), ("fp32", P.PIC_FP32)):
        log(f"precision: 10,000-cell instance against the oracle, {name} form")
        sim = P.PicSim(wl, None, prec, capacities=gold["caps"], flags=P.PIC_INIT_DEVICE)
        rows, last = [], 0
        for c in checks:
            sim.step_graph(c - last, SORT_EVERY)
            last = c
            rows.append(_gpu_moments(torch, sim, wl.nc, bins))
        runs[name] = rows
        sim.close()
    out["subsample_vs_oracle"] = [
        {"step": c, "fp64_vs_oracle": _rel_diff(runs["fp64"][i], gold["moments"][i + 1]),
         "fp32_vs_oracle": _rel_diff(runs["fp32"][i], gold["moments"][i + 1])}
        for i, c in enumerate(checks)]
    # ---- the precision configuration: 1,000,000 cells, 4e8 particles
    wl = pin.bounded_mcc(nc=args.precision_cells, ppc=200, seed=5)
    n = wl.n_particles
    caps = [int(0.75 * n) + 1024] * 2  # ionisation grows the plasma by about 25% in 2,000 steps
    out["large"] = {"cells": wl.nc, "particles": n}
    out["large"].update(precision_protocol(torch, wl, caps, args.precision_steps, args.precision_K,
                                           P.PIC_INIT_DEVICE | P.PIC_INIT_SORT,
                                           f" ({wl.nc} cells)"))
    return out


def layout_study(torch, args):
    """The mover pass in four particle layouts (libpic_layout): structure of
    arrays (libpic's), array of 32-byte structs, 64-particle blocks of arrays,
    and per-cell slots with slack regrouped every pass (natural sorting).  One
    magnetised species of 2e7 particles on 100,000 periodic cells (200 per
    cell, B at 45 degrees with |t| = 0.1, v_th = 0.05 cells/step, 4.6%
    candidates), drawn on the device in cell order; each layout is timed with
    HIP events over `passes` passes after 5 warm-up passes."""
    from paper_2404_10270_amd import layout as Lb
    nc, ppc, passes = 100_000, 200, args.layout_passes
    n = nc * ppc
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    x = torch.sort(torch.rand(n, generator=g, device=dev, dtype=torch.float64) * nc).values
    cell = torch.floor(x).to(torch.int32)
    f = (x - cell.to(torch.float64)).to(torch.float32)
    f = torch.where(f >= 1.0, torch.full_like(f, 0.99999994), f)
    del x
    v = torch.randn(3, n, generator=g, device=dev, dtype=torch.float32) * 0.05
    soa = {"cell": cell, "f": f, "vx": v[0].contiguous(), "vy": v[1].contiguous(),
           "vz": v[2].contiguous(), "id": torch.arange(n, dtype=torch.int64, device=dev)}
    del v
    acc = (1e-4 * torch.sin(2 * math.pi * torch.arange(nc + 1, device=dev, dtype=torch.float64) / nc)
           ).to(torch.float32)
    S = torch.zeros(nc + 1, dtype=torch.int64, device=dev)
    per_cell = int(torch.bincount(cell, minlength=nc).max())
    slack = int(math.ceil(per_cell * 1.5 / 64.0) * 64)
    tm = 0.1
    tx = ty = tm * math.cos(math.pi / 4)
    den = 1.0 + (tx * tx + ty * ty)
    p = Lb.pls_params()
    p.nc, p.slack = nc, slack
    p.tx, p.ty, p.sx, p.sy = tx, ty, 2 * tx / den, 2 * ty / den
    p.key0, p.key1 = 3, 0
    p.T = int(math.floor(-math.expm1(-0.047) * 2 ** 32))
    p.acc, p.S = acc.data_ptr(), S.data_ptr()
    out = {"particles": n, "cells": nc, "passes": passes, "slack": slack,
           "bytes_per_particle": 48}
    for name, lay in Lb.LAYOUTS.items():
        log(f"layout study: {name}")
        r = Lb.LayoutRun(lay, soa, nc, slack)
        for s in range(5):
            r.step(p, s)
        st = r.stream
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for s in range(passes):
            r.step(p, 5 + s)
        e1.record(st)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / passes
        _, n_cand = r.store()
        foot = (r.work.numel() - 256) / n
        out[name] = {"us_per_pass": round(us, 1), "particle_steps_per_s": n / (us * 1e-6),
                     "GBps": round(48 * n / (us * 1e-6) / 1e9, 1),
                     "frac": round(48 * n / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "bytes_stored_per_particle": round(foot, 1), "candidates": n_cand}
        log(f"layout study: {name} {us:.1f} us/pass, {out[name]['GBps']} GB/s, "
            f"{foot:.1f} B stored per particle")
        del r
        torch.cuda.empty_cache()
    return out


def small_configs(torch, args):
    """The two small configurations, both drawn on the device and replayed
    from a HIP graph: the periodic Langmuir plasma (512 cells, 51,200
    electrons, FP64, its 200 steps, no sort) and the bounded magnetised plasma
    (8,192 cells, 200 particles per cell per species, FP32, B at 45 degrees,
    pair source, no collisions, sort every 20 steps, 200 steps after 20).
    Their state fits in the 256 MB last-level cache, so they measure launch
    and latency, not HBM."""
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P
    out = {}
    wl = pin.langmuir()
    sim = P.PicSim(wl, None, P.PIC_FP64, flags=P.PIC_INIT_DEVICE)
    sim.step_graph(0, 0)  # the one-step graph, captured untimed
    d0, _ = sim.diagnostics()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step_graph(wl.n_steps, 0)
    e1.record(sim.stream)
    d1, rc = sim.diagnostics()
    if rc != 0:
        raise RuntimeError(f"device status {d1[0].status:#x} in the Langmuir run")
    ms = e0.elapsed_time(e1)
    ps = int(d1[0].particle_steps - d0[0].particle_steps)
    sim.close()
    out["langmuir_512_cells_fp64"] = {"value": ps / (ms * 1e-3), "unit": "particle-steps/s",
                                      "particles": wl.n_particles, "steps": wl.n_steps,
                                      "ms_per_step": round(ms / wl.n_steps, 4)}
    log(f"langmuir: {ps / (ms * 1e-3):.4e} p-steps/s, {ms / wl.n_steps:.4f} ms/step")
    wl = pin.bounded()
    sim = P.PicSim(wl, None, P.PIC_FP32, flags=P.PIC_INIT_DEVICE | P.PIC_INIT_SORT)
    rate, ms_step, _ = run_form(torch, sim, 200, 20, graph=True)
    win = time_windows(torch, sim)
    sim.close()
    out["bounded_8192_cells_fp32"] = {"value": rate, "unit": "particle-steps/s",
                                      "particles": wl.n_particles, "steps": 200,
                                      "ms_per_step": round(ms_step, 4), "windows": win}
    log(f"bounded 8192 cells: {rate:.4e} p-steps/s, {ms_step:.4f} ms/step")
    return out


def large_run(torch, args):
    """The largest single-GPU configuration: the collisional bounded plasma on
    1,000,000 cells with 200 particles per cell per species (4e8 particles),
    drawn on the device and sorted, sort every 20 steps, as the FP32/fixed-point
    form and as the FP64 form: whole steps from the HIP graph, five one-period
    windows, and the mover's algorithmic bandwidth from HIP events."""
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P
    wl = pin.bounded_mcc(nc=args.large_cells, ppc=200, seed=5, sort_every=SORT_EVERY)
    n = wl.n_particles
    caps = [int(0.55 * n) + 1024] * 2
    out = {"cells": wl.nc, "particles": n, "steps": args.large_steps, "sort_every": SORT_EVERY}
    for name, prec, bpp in (("fp32", P.PIC_FP32, PUSH_BYTES_FP32), ("fp64", P.PIC_FP64, PUSH_BYTES_FP64)):
        log(f"large: {wl.nc} cells, {n} particles, {name} form")
        sim, mv = tuned_sim(torch, lambda: P.PicSim(wl, None, prec, capacities=caps,
                                                    flags=P.PIC_INIT_DEVICE | P.PIC_INIT_SORT))
        log(f"large {name}: autotuned mover {mv}")
        rate, ms_step, _ = run_form(torch, sim, args.large_steps, args.warmup, graph=True)
        win = time_windows(torch, sim)
        push_ms, per_launch = time_push(torch, sim, 10)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        gbs = bpp * per_launch / (push_ms * 1e-3) / 1e9
        out[name] = {"value": rate, "ms_per_step": round(ms_step, 4), "windows": win, "mover": mv,
                     "mover_us": round(push_ms * 1e3, 1), "mover_GBps": round(gbs, 1),
                     "mover_frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_particle": bpp}
        log(f"large {name}: {rate:.4e} p-steps/s, {ms_step:.4f} ms/step, mover {push_ms * 1e3:.1f} us "
            f"({gbs:.0f} GB/s)")
    out["fp32_over_fp64"] = round(out["fp32"]["value"] / out["fp64"]["value"], 3)
    return out


def host_info():
    """CPU model, logical CPUs, the CPUs this process may run on, and the
    threads the CPU baseline uses (OMP_NUM_THREADS when set, else all)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(int(omp), avail) if omp.isdigit() and int(omp) > 0 else avail
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail,
            "threads": threads}


def cpu_baseline(args):
    """The oracle as it stands on the host's cores: `cpu_steps` whole steps of
    the bench workload from its seeded start, on every available thread (the
    oracle's independent per-particle loops in parallel, results bit-identical
    to one thread) and on one thread."""
    import oracle
    import pic_inputs as pin
    host = host_info()
    wl = workload(args)
    st = pin.initial_state(wl)
    st32 = pin.to_fp32_form(st, wl.nc)
    st_o = [s.as_f64() for s in st32]
    del st, st32
    caps = pin.capacities(wl, st_o)
    n = sum(s.n for s in st_o)
    ps, dt = oracle.time_steps(wl, st_o, args.cpu_steps, caps=caps, n_threads=host["threads"])
    ps1, dt1 = oracle.time_steps(wl, st_o, args.cpu_steps, caps=caps, n_threads=1)
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": host["threads"], "kind": "oracle",
            "sample": f"{wl.nc} cells, {n} particles, {args.cpu_steps} whole steps from the seeded "
                      f"start: {dt:.1f} s on {host['threads']} threads, {dt1:.1f} s on one",
            "single_thread": {"value": ps1 / dt1, "seconds": round(dt1, 2)},
            "host": host}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nc", type=int, default=100_000)
    ap.add_argument("--ppc", type=float, default=100)
    ap.add_argument("--push-steps", type=int, default=40)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-instances", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=60)
    ap.add_argument("--no-table1", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-cells", type=int, default=1_000_000)
    ap.add_argument("--large-steps", type=int, default=20)
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--table1-steps", type=int, default=200)
    ap.add_argument("--layout-study", action="store_true",
                    help="run only the particle-layout study of the mover and print its JSON object")
    ap.add_argument("--layout-passes", type=int, default=40)
    ap.add_argument("--precision-study", action="store_true",
                    help="FP32 form against FP64 form and the oracle (1e6- and 1e4-cell instances); prints its own JSON")
    ap.add_argument("--precision-cells", type=int, default=1_000_000)
    ap.add_argument("--precision-steps", type=int, default=2000)
    ap.add_argument("--precision-K", type=int, default=8,
                    help="perturbed FP64 runs in the ensemble of the large instance")
    ap.add_argument("--precision-skip-small", action="store_true",
                    help="skip the 10^4-step protocol on the 10,000-cell instance (the GPU test runs it)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched workload and print its JSON object (profiling)")
    ap.add_argument("--only-table1", action="store_true",
                    help="run only the Table 1 workload and print its JSON object (profiling)")
    ap.add_argument("--eager", action="store_true",
                    help="enqueue the timed steps one by one instead of replaying a HIP graph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to scale the HBM byte counters")
    ap.add_argument("--pmc-summary", nargs=5, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE", "OUT"),
                    help="summarise four rocprofv3 --pmc CSV directories into OUT (no GPU)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    import pic_inputs as pin
    from paper_2404_10270_amd import pic as P

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.layout_study:
        print(json.dumps({"layout_study": layout_study(torch, args)}), flush=True)
        return
    if args.precision_study:
        print(json.dumps({"precision_study": precision_study(torch, args)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps(batched(torch, args)), flush=True)
        return
    if args.only_table1:
        print(json.dumps(table1_run(torch, args)), flush=True)
        return
    wl = workload(args)
    log(f"generating {wl.n_particles} particles on {wl.nc} cells")
    st = pin.initial_state(wl)

    log("FP32 form: init")
    sim, mover32 = tuned_sim(torch, lambda: make_sim(wl, st, P.PIC_FP32))
    log(f"FP32 form: autotuned mover {mover32}")
    log(f"FP32 form: {args.warmup} warm-up + {args.steps} timed steps")
    rate, ms_step, ps = run_form(torch, sim, args.steps, args.warmup, graph=not args.eager)
    log(f"FP32 form: {rate:.4e} p-steps/s, {ms_step:.4f} ms/step")
    win = time_windows(torch, sim)
    log(f"FP32 form: windows median {win['median']:.4e} ({win['min']:.4e} .. {win['max']:.4e})")
    push_ms, per_launch = time_push(torch, sim, args.push_steps)
    log(f"FP32 mover: {push_ms * 1e3:.1f} us/launch, {per_launch:.0f} particles/launch")
    sim.close()
    del sim
    torch.cuda.empty_cache()

    achieved = PUSH_BYTES_FP32 * per_launch / (push_ms * 1e-3) / 1e9
    copy_gbs = copy_rate(torch)
    log(f"plain copy: {copy_gbs:.0f} GB/s (mover at {achieved / copy_gbs:.2f} of it)")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(),
            "kernel": f"{MOVER_KERNEL} (mover + deposit + candidate list, as pic_push launches it; "
                      f"timed at the autotuned grid of {mover32['blocks']} blocks)",
            "mover": mover32,
            "bytes_per_particle": PUSH_BYTES_FP32,
            "particles_per_launch": int(per_launch), "us_per_launch": round(push_ms * 1e3, 2),
            "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}

    fp64 = None
    if not args.no_fp64:
        log("FP64 form: init")
        sim64, mover64 = tuned_sim(torch, lambda: make_sim(wl, st, P.PIC_FP64))
        log(f"FP64 form: autotuned mover {mover64}")
        r64, ms64, _ = run_form(torch, sim64, args.steps, args.warmup, graph=not args.eager)
        win64 = time_windows(torch, sim64)
        p64_ms, per64 = time_push(torch, sim64, args.push_steps)
        log(f"FP64 form: {r64:.4e} p-steps/s, mover {p64_ms * 1e3:.1f} us")
        g64 = PUSH_BYTES_FP64 * per64 / (p64_ms * 1e-3) / 1e9
        fp64 = {"value": r64, "ms_per_step": round(ms64, 4), "windows": win64,
                "mover_us": round(p64_ms * 1e3, 2), "mover_GBps": round(g64, 1),
                "mover_frac": round(g64 / HBM_PEAK_GBS, 4), "mover": mover64,
                "fp32_over_fp64": round(rate / r64, 3)}
        sim64.close()
        del sim64
        torch.cuda.empty_cache()

    bat = None
    if not args.no_batched:
        bat = batched(torch, args)
        torch.cuda.empty_cache()

    t1 = None
    if not args.no_table1:
        t1 = table1_run(torch, args)
        torch.cuda.empty_cache()

    small = None
    if not args.no_small:
        small = small_configs(torch, args)
        torch.cuda.empty_cache()

    large = None
    if not args.no_large:
        large = large_run(torch, args)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU baseline: oracle, {args.cpu_steps} steps")
        cpu = cpu_baseline(args)
        log(f"CPU baseline: {cpu['value']:.4e} p-steps/s")

    out = {
        "metric": "particle-steps/s on 1 MI355X",
        "value": rate,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "bounded plasma + null-collision MCC, 100,000 cells, "
                               "100 particles/cell/species",
                   "cells": wl.nc, "particles": wl.n_particles, "sort_every": SORT_EVERY,
                   "deposit": "int64 fixed point (F=32)", "field_solve": "f64 Thomas",
                   "launch": "eager" if args.eager else "hip graph (pic_step_graph)"},
        "windows": win,
        "roofline": roof,
        "fp64_form": fp64,
        "large_1e6_cells": large,
        "small_configs": small,
        "batched_256": bat,
        "table1": t1,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
