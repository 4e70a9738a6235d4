"""Pins of the oracle's subcycling (the per-species step multiplier nstep of
the moveb listing, Sec. 6): a species with nstep = m moves only on steps
s with s mod m = 0, over m dt.  Closed forms: its gyration angle per push is
2 atan(omega_c m dt / 2) with |v| conserved; with a uniform acceleration a
along B the velocity grows by m a per push and the position by m v; between
pushes nothing changes; its collision test runs on push steps only, with the
null-collision probability of m dt."""
import math

import numpy as np
import pytest

import pic_inputs as pin


def _single(oracle_lib, x, v, nstep, B0=0.0, theta=0.0, nc=64, bc=pin.BC_PERIODIC):
    sp = [pin.Species("i", pin.KIND_ION, q=1.0, m=1.0, w=1.0, ppc=0, T=0, nstep=nstep)]
    wl = pin.Workload(name="t", nc=nc, bc=bc, dx=1.0, dt=1.0, eps0=1.0, species=sp, B0=B0,
                      theta=theta)
    st = [pin.SpeciesState(x=np.array(x, float), vx=np.array([v[0]], float),
                           vy=np.array([v[1]], float), vz=np.array([v[2]], float),
                           id=np.zeros(1, np.uint64))]
    return oracle_lib.OracleSim(wl, st, caps=[1])


def _v(o):
    return np.array([o.vx[0][0], o.vy[0][0], o.vz[0][0]])


@pytest.mark.parametrize("m", [2, 4, 7])
def test_subcycled_gyration(oracle_lib, m):
    wc_dt = 0.05
    th = math.radians(35.0)
    o = _single(oracle_lib, [10.5], (0.01, -0.02, 0.015), m, B0=wc_dt, theta=th)
    bhat = np.array([math.cos(th), math.sin(th), 0.0])
    v0 = _v(o)
    expect = 2.0 * math.atan(wc_dt * m / 2.0)
    prev = v0 - bhat * v0.dot(bhat)
    x_prev = o.x[0][0]
    for s in range(6 * m):
        o.sim.cnt.step = s
        o.push()
        v = _v(o)
        vperp = v - bhat * v.dot(bhat)
        if s % m:
            assert np.array_equal(vperp, prev) and o.x[0][0] == x_prev
            continue
        assert abs(np.linalg.norm(v) - np.linalg.norm(v0)) <= 1e-15 * 6 * np.linalg.norm(v0)
        ang = math.atan2(np.linalg.norm(np.cross(prev, vperp)), prev.dot(vperp))
        assert abs(ang - expect) <= 1e-12
        prev, x_prev = vperp, o.x[0][0]


@pytest.mark.parametrize("m", [1, 3, 8])
def test_subcycled_kick_and_advance_exact(oracle_lib, m):
    """B along x (theta = 0) with uniform a: v_N = v0 + N m a and
    x_N = x0 + m (N v0 + m a N (N + 1) / 2), exactly for dyadic inputs."""
    a, v0, x0 = 2.0 ** -12, 2.0 ** -7, 100.25
    o = _single(oracle_lib, [x0], (v0, 0.0, 0.0), m, B0=0.1, theta=0.0, nc=1024,
                bc=pin.BC_ABSORB)
    o.acc[0][:] = a
    n_push = 0
    for s in range(9 * m):
        o.sim.cnt.step = s
        o.push()
        n_push += (s % m == 0)
        assert o.vx[0][0] == v0 + n_push * m * a
        assert o.x[0][0] == x0 + m * (n_push * v0 + m * a * n_push * (n_push + 1) / 2)


def test_subcycled_collisions_on_push_steps_only(oracle_lib):
    wl = pin.bounded_mcc(nc=400, ppc=250, seed=13)
    wl.species[1].nstep = 3
    st = pin.initial_state(wl)
    o = oracle_lib.OracleSim(wl, st)
    cx = [0]
    for s in range(9):
        o.step(1)
        cx.append(o.counters.n_cx)
    grow = np.diff(cx)
    assert np.all(grow[[1, 2, 4, 5, 7, 8]] == 0)
    assert np.all(grow[[0, 3, 6]] > 0)
    # the candidate probability per push is that of 3 dt: 1 - exp(-3 nu) = 1 - (1 - P1)^3
    P3 = o.candidate_threshold(1) / 2.0 ** 32
    o1 = oracle_lib.OracleSim(pin.bounded_mcc(nc=400, ppc=250, seed=13), st)
    P1 = o1.candidate_threshold(1) / 2.0 ** 32
    assert abs(P3 - (1.0 - (1.0 - P1) ** 3)) <= 2e-9


def test_particle_steps_count_pushes(oracle_lib):
    wl = pin.bounded(nc=200, ppc=20, seed=14, source=False)
    wl.species[1].nstep = 4
    st = pin.initial_state(wl)
    o = oracle_lib.OracleSim(wl, st)
    o.step(8)
    n_e, n_i = st[0].n, st[1].n
    # absorption is negligible in 8 steps of this plasma; ions are pushed on steps 0 and 4
    assert abs(o.counters.particle_steps - (8 * n_e + 2 * n_i)) <= 0.01 * n_e
