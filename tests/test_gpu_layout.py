"""The layout study (libpic_layout): its mover pass in every layout computes
libpic's FP32 mover bit for bit.

* one pass of each layout against libpic's own FP32 push (pic_push) of the
  same particles on the same grid acceleration: cell, offset and velocity
  identical for every particle (by id);
* five passes: every layout identical to the structure-of-arrays one, the
  fixed-point deposits identical, the candidate counts identical;
* the cell-padded layout returns the particles grouped by cell.
"""
import math

import numpy as np
import pytest

import pic_inputs as pin
from gpu_common import FP32, P, flush

pytestmark = pytest.mark.gpu


def _setup(nc=300, ppc=100, seed=51):
    import torch
    wl = pin.bounded(nc=nc, ppc=ppc, seed=seed, source=False).replace(bc=pin.BC_PERIODIC,
                                                                      pair_start=False)
    wl = wl.replace(species=[wl.species[0]])
    st = pin.to_fp32_form(pin.initial_state(wl), wl.nc)
    rng = np.random.default_rng(seed)
    acc64 = 1e-4 * np.sin(2 * np.pi * np.arange(wl.nc + 1) / wl.nc) + 1e-5 * rng.standard_normal(wl.nc + 1)
    acc64[-1] = acc64[0]
    s = st[0]
    dev = torch.device("cuda")
    soa = {"cell": torch.from_numpy(s.cell.astype(np.int32)).to(dev),
           "f": torch.from_numpy(s.f.astype(np.float32)).to(dev),
           "vx": torch.from_numpy(s.vx.astype(np.float32)).to(dev),
           "vy": torch.from_numpy(s.vy.astype(np.float32)).to(dev),
           "vz": torch.from_numpy(s.vz.astype(np.float32)).to(dev),
           "id": torch.from_numpy(s.id.view(np.int64)).to(dev)}
    return wl, st, acc64, soa


def _params(wl, acc32, S, T=0):
    from paper_2404_10270_amd import layout as Lb
    sp = wl.species[0]
    # the rotation vectors as libpic forms them (FP64, then rounded to FP32)
    tm = (sp.q / sp.m) * wl.B0 * (0.5 * (wl.dt * 1.0))
    tx, ty = tm * math.cos(wl.theta), tm * math.sin(wl.theta)
    den = 1.0 + (tx * tx + ty * ty)
    p = Lb.pls_params()
    p.nc, p.slack = wl.nc, 0
    p.tx, p.ty = float(np.float32(tx)), float(np.float32(ty))
    p.sx, p.sy = float(np.float32(2.0 * tx / den)), float(np.float32(2.0 * ty / den))
    p.key0, p.key1 = 0x1234, 0x5678
    p.T = T
    p.acc = acc32.data_ptr()
    p.S = S.data_ptr()
    return p


def _np(d):
    o = np.argsort(d["id"].cpu().numpy(), kind="stable")
    return {k: v.cpu().numpy()[o] for k, v in d.items()}


def _slack(wl, st):
    per_cell = np.bincount(st[0].cell, minlength=wl.nc).max()
    return int(math.ceil(per_cell * 1.5 / 64.0) * 64)


def test_one_pass_equals_libpic_fp32_push():
    import torch
    from paper_2404_10270_amd import layout as Lb
    wl, st, acc64, soa = _setup()
    flush("layout study: one pass vs pic_push")
    sim = P.PicSim(wl, st, FP32, flags=P.PIC_INIT_NO_FIELD)
    sim.set_acc([acc64])
    sim.push(P.PIC_PUSH_NO_DEPOSIT)
    ref = sim.state(0)
    o = np.argsort(ref["id"], kind="stable")
    ref = {k: (v[o] if isinstance(v, np.ndarray) and v.shape == ref["id"].shape else v) for k, v in ref.items()}
    sim.close()
    acc32 = torch.from_numpy(acc64.astype(np.float32)).cuda()
    slack = _slack(wl, st)
    for name, lay in Lb.LAYOUTS.items():
        S = torch.zeros(wl.nc + 1, dtype=torch.int64, device="cuda")
        r = Lb.LayoutRun(lay, {k: v.clone() for k, v in soa.items()}, wl.nc, slack)
        p = _params(wl, acc32, S)
        p.slack = slack
        r.step(p, step=0)
        out, _ = r.store()
        g = _np(out)
        assert np.array_equal(g["id"].view(np.uint64), ref["id"]), name
        xg = g["cell"].astype(np.float64) + g["f"].astype(np.float64)
        assert np.array_equal(xg, ref["x"]), f"{name}: positions differ"
        for f in ("vx", "vy", "vz"):
            assert np.array_equal(g[f].astype(np.float64), ref[f]), f"{name}: {f} differs"


def test_layouts_agree_over_five_passes():
    import torch
    from paper_2404_10270_amd import layout as Lb
    wl, st, acc64, soa = _setup(nc=500, ppc=80, seed=52)
    flush("layout study: five passes, all layouts")
    acc32 = torch.from_numpy(acc64.astype(np.float32)).cuda()
    slack = _slack(wl, st)
    res = {}
    for name, lay in Lb.LAYOUTS.items():
        S = torch.zeros(wl.nc + 1, dtype=torch.int64, device="cuda")
        r = Lb.LayoutRun(lay, {k: v.clone() for k, v in soa.items()}, wl.nc, slack)
        p = _params(wl, acc32, S, T=int(0.05 * 2 ** 32))
        p.slack = slack
        for s in range(5):
            r.step(p, step=s)
        out, n_cand = r.store()
        torch.cuda.synchronize()
        res[name] = (_np(out), S.cpu().numpy().view(np.uint64), n_cand, out)
    base, S0, c0, _ = res["soa"]
    assert int(S0.sum(dtype=np.uint64)) == 5 * base["id"].size * 2 ** 32
    assert 0.04 * 5 * base["id"].size < c0 < 0.06 * 5 * base["id"].size
    for name, (g, S, c, raw) in res.items():
        for f in ("id", "cell", "f", "vx", "vy", "vz"):
            assert np.array_equal(g[f], base[f]), f"{name}: {f}"
        assert np.array_equal(S, S0), f"{name}: deposit"
        assert c == c0, f"{name}: candidates"
    # natural sorting hands the particles back grouped by cell
    cells = res["cellpad"][3]["cell"].cpu().numpy()
    assert np.all(np.diff(cells) >= 0)


def test_one_pass_of_every_layout_against_the_oracle():
    """One pass of each layout against the oracle's FP64 push of the same
    particles on the same grid acceleration (Sec. 6 moveb statements with the
    Boris rotation): positions within 1e-5 cells and velocities within
    1e-5 max(|v|, v_th) (FP32 tolerance); the pass's fixed-point deposit of its
    new positions bit-exact against the oracle's deposit of those positions;
    the candidate count equal to the oracle Philox draws of the same ids."""
    import torch

    import oracle
    from paper_2404_10270_amd import layout as Lb
    wl, st, acc64, soa = _setup(nc=400, ppc=100, seed=53)
    flush("layout study: one pass of each layout vs the oracle")
    ost = [s.as_f64() for s in st]
    orc = oracle.OracleSim(wl, ost, caps=[ost[0].n + 1])
    orc.acc[0][:] = acc64
    orc.push()
    orc.walls()
    o = orc.state(0)
    order = np.argsort(o.id, kind="stable")
    o_id, o_x = o.id[order], o.x[order]
    o_v = {f: getattr(o, f)[order] for f in ("vx", "vy", "vz")}
    vth = wl.vth_hat(wl.species[0])
    T = int(0.05 * 2 ** 32)
    key0, key1 = 0x1234, 0x5678
    n_cand = sum(int(oracle.philox4x32_10([int(i) & 0xFFFFFFFF, int(i) >> 32, 0, 0], [key0, key1])[0]) < T
                 for i in ost[0].id)
    acc32 = torch.from_numpy(acc64.astype(np.float32)).cuda()
    slack = _slack(wl, st)
    for name, lay in Lb.LAYOUTS.items():
        S = torch.zeros(wl.nc + 1, dtype=torch.int64, device="cuda")
        r = Lb.LayoutRun(lay, {k: v.clone() for k, v in soa.items()}, wl.nc, slack)
        p = _params(wl, acc32, S, T=T)
        p.slack = slack
        r.step(p, step=0)
        out, c = r.store()
        g = _np(out)
        assert np.array_equal(g["id"].view(np.uint64), o_id), name
        xg = g["cell"].astype(np.float64) + g["f"].astype(np.float64)
        dxw = np.abs(xg - o_x)
        dxw = np.minimum(dxw, wl.nc - dxw)  # positions on a ring
        assert np.max(dxw) <= 1e-5, f"{name}: positions {np.max(dxw)}"
        for f in ("vx", "vy", "vz"):
            err = np.abs(g[f].astype(np.float64) - o_v[f]) / np.maximum(np.abs(o_v[f]), vth)
            assert np.max(err) <= 1e-5, f"{name}: {f} {np.max(err)}"
        S_ref = oracle.deposit_fixed(xg, wl.nc)
        assert np.array_equal(S.cpu().numpy().view(np.uint64), S_ref), f"{name}: deposit"
        assert c == n_cand, f"{name}: candidates {c} vs {n_cand}"
