"""The oracle on several threads (the all-core CPU baseline) computes exactly
what it computes on one: the same particles in the same order, counters,
deposit, field and diagnostics, bit for bit, on a collisional bounded plasma
with walls, ionisation and source, on the periodic Langmuir case, and on the
Table 1 case with kinetic atoms."""
import ctypes as C

import numpy as np
import pytest

import oracle
import pic_inputs as pin


def _run(wl, st, caps, steps, n_threads):
    prev = oracle.threads()
    oracle.set_threads(n_threads)
    try:
        o = oracle.OracleSim(wl, st, caps=caps)
        o.step(steps)
        d = o.diagnostics()
    finally:
        oracle.set_threads(prev)
    return o, d


def _same(a, b, nsp):
    oa, da = a
    ob, db = b
    assert bytes(oa.sim.cnt) == bytes(ob.sim.cnt)
    assert bytes(da) == bytes(db)
    for k in range(nsp):
        sa, sb = oa.state(k), ob.state(k)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(getattr(sa, f), getattr(sb, f)), (k, f)
        assert np.array_equal(oa.S[k], ob.S[k]) and np.array_equal(oa.acc[k], ob.acc[k]), k
    for f in ("rho", "phi", "E", "nn"):
        assert np.array_equal(getattr(oa, f), getattr(ob, f)), f


@pytest.mark.parametrize("case", ["bounded_mcc", "langmuir", "table1"])
def test_threads_give_bit_identical_results(case):
    if case == "bounded_mcc":
        wl = pin.bounded_mcc(nc=3000, ppc=40, seed=12)
        wl.mcc.n_n *= 20  # many collisions and ionisation pairs per step
        steps = 25
    elif case == "langmuir":
        wl = pin.langmuir()
        steps = 30
    else:
        base = pin.table1(nc=400, ppc=40, L=400e-5, seed=13)
        sig = 0.2 / (4e21 * base.species[0].v_cap * base.dt)
        wl = base.replace(mcc=pin.MCC(n_n=4e21, T_n=pin.EV, sig_el=0.3 * sig, sig_ex=0.2 * sig,
                                      E_ex=10.2 * pin.EV, sig_iz=0.5 * sig, E_iz=13.6 * pin.EV,
                                      sig_cx=0.0))
        steps = 12
    st = pin.initial_state(wl)
    caps = [s.n * 3 + 4096 for s in st]
    one = _run(wl, st, caps, steps, 1)
    many = _run(wl, st, caps, steps, 4)
    assert oracle.threads() == 1
    _same(one, many, len(wl.species))
    # something happened: particles moved, and in the collisional cases collided
    assert one[0].sim.cnt.particle_steps > 0
    if case != "langmuir":
        assert one[0].sim.cnt.n_candidates > 0 and one[0].sim.cnt.n_ionize > 0
