"""Pins of the oracle's mover (Sec. 2 phase 5 and the moveb listing of Sec. 6:
linear gather in the in-cell coordinate, velocity kick, advance x += vx),
extended to a magnetised Boris rotation for the 1D3V case.

Closed forms used: gyration of a single particle (|v| conserved, rotation by
2 atan(omega_c dt / 2) per step), the E x B drift and the exact parallel
acceleration of the Boris scheme, the reduction to 1D leapfrog when B is
along x, and the cold Langmuir frequency of leapfrog,
omega = (2/dt) asin(omega_p dt / 2).
"""
import math

import numpy as np
import pytest

import pic_inputs as pin


def _single(oracle_lib, x, v, B0=0.0, theta=0.0, q=-1.0, m=1.0, dt=1.0, nc=64,
            bc=pin.BC_PERIODIC):
    sp = [pin.Species("e", pin.KIND_ELECTRON, q=q, m=m, w=1.0, ppc=0, T=0)]
    wl = pin.Workload(name="t", nc=nc, bc=bc, dx=1.0, dt=dt, eps0=1.0, species=sp,
                      B0=B0, theta=theta)
    n = len(x)
    st = [pin.SpeciesState(x=np.array(x, dtype=float), vx=np.array([vv[0] for vv in v], float),
                           vy=np.array([vv[1] for vv in v], float),
                           vz=np.array([vv[2] for vv in v], float),
                           id=np.arange(n, dtype=np.uint64))]
    return oracle_lib.OracleSim(wl, st, caps=[n])


@pytest.mark.parametrize("theta_deg", [0.0, 30.0, 45.0, 85.0])
def test_gyration_angle_and_speed(oracle_lib, theta_deg):
    wc_dt = 0.2
    th = math.radians(theta_deg)
    o = _single(oracle_lib, [10.5], [(0.03, 0.02, -0.01)], B0=wc_dt, theta=th, q=-1.0, m=1.0)
    bhat = np.array([math.cos(th), math.sin(th), 0.0])
    v0 = np.array([o.vx[0][0], o.vy[0][0], o.vz[0][0]])
    vperp0 = v0 - bhat * v0.dot(bhat)
    expect = 2.0 * math.atan(wc_dt / 2.0)
    assert abs(expect - 0.19933730) < 1e-8
    prev = vperp0
    for _ in range(25):
        o.push()  # acc arrays are zero: no electric field
        o.walls()
        v = np.array([o.vx[0][0], o.vy[0][0], o.vz[0][0]])
        assert abs(np.linalg.norm(v) - np.linalg.norm(v0)) <= 4e-16 * np.linalg.norm(v0) * 25
        vperp = v - bhat * v.dot(bhat)
        assert abs(v.dot(bhat) - v0.dot(bhat)) <= 2e-15 * np.linalg.norm(v0)
        ang = math.atan2(np.linalg.norm(np.cross(prev, vperp)), prev.dot(vperp))
        assert abs(ang - expect) <= 1e-12
        prev = vperp


@pytest.mark.parametrize("theta_deg", [20.0, 45.0, 70.0])
def test_exb_drift_and_parallel_acceleration(oracle_lib, theta_deg):
    """Uniform E_x with B at theta: in the frame moving with v_E = E_x sin(th)/B z,
    the perpendicular velocity only rotates; v_par grows by (q/m) E_x cos(th) dt."""
    wc_dt = 0.3
    th = math.radians(theta_deg)
    o = _single(oracle_lib, [20.25], [(0.0, 0.0, 0.0)], B0=wc_dt, theta=th, nc=200,
                bc=pin.BC_ABSORB)
    a = 1e-4  # acc = (q/m) E dt^2/dx, uniform
    o.acc[0][:] = a
    tmag = (-1.0) * wc_dt * 0.5  # t = (q/m) B dt / 2, signed
    bhat = np.array([math.cos(th), math.sin(th), 0.0])
    vE = np.array([0.0, 0.0, (a / (2.0 * tmag)) * math.sin(th)])
    v_prev_par = 0.0
    radii = []
    for _ in range(60):
        o.push()
        v = np.array([o.vx[0][0], o.vy[0][0], o.vz[0][0]])
        vpar = v.dot(bhat)
        assert abs((vpar - v_prev_par) - a * math.cos(th)) <= 1e-15
        v_prev_par = vpar
        w = v - bhat * vpar - vE
        radii.append(np.linalg.norm(w))
    radii = np.array(radii)
    assert np.max(np.abs(radii - radii[0])) <= 1e-13 * np.max(np.abs(vE))


def test_b_along_x_is_plain_leapfrog(oracle_lib):
    """theta = 0: the x motion is the unmagnetised 1D leapfrog (vx += a, x += vx)."""
    o = _single(oracle_lib, [5.5], [(0.01, 0.02, 0.03)], B0=0.4, theta=0.0, nc=100)
    o.acc[0][:] = np.linspace(0, 1e-3, 101)
    x, vx = 5.5, 0.01
    for _ in range(30):
        j = math.floor(x)
        f = x - j
        a = o.acc[0][j] + f * (o.acc[0][j + 1] - o.acc[0][j])
        vx = vx + a
        x = x + vx
        o.push()
        assert abs(o.vx[0][0] - vx) <= 1e-15
        assert abs(o.x[0][0] - x) <= 1e-13


def test_linear_gather_endpoints(oracle_lib):
    """The gather returns a[j] at f = 0 and interpolates linearly inside the cell."""
    o = _single(oracle_lib, [3.0, 3.5, 3.75], [(0, 0, 0)] * 3, nc=10)
    o.acc[0][:] = np.arange(11) * 0.01
    o.push()
    # vx = 0 + a (no B): a at x = 3, 3.5, 3.75 -> 0.03, 0.035, 0.0375
    assert np.allclose(o.vx[0][:3], [0.03, 0.035, 0.0375], rtol=0, atol=1e-17)


def _mode1_amplitude(E, nc):
    j = np.arange(nc)
    return np.sum(E[:nc] * np.sin(2 * math.pi * j / nc))


def test_cold_langmuir_frequency(oracle_lib):
    """Quiet cold start: the mode-1 field oscillates at (2/dt) asin(omega_p dt/2)."""
    wl = pin.langmuir(quiet=True, n_steps=800)
    st = pin.initial_state(wl)
    o = oracle_lib.OracleSim(wl, st)
    amps = []
    for _ in range(wl.n_steps):
        o.step(1)
        amps.append(_mode1_amplitude(o.E, wl.nc))
    amps = np.array(amps)
    t = np.arange(len(amps), dtype=float)
    # least-squares fit of A cos(w t) + B sin(w t) over w
    def resid(w):
        M = np.stack([np.cos(w * t), np.sin(w * t)], axis=1)
        c, *_ = np.linalg.lstsq(M, amps, rcond=None)
        return np.sum((M @ c - amps) ** 2)
    ws = np.linspace(0.095, 0.105, 2001)
    r = np.array([resid(w) for w in ws])
    i = int(np.argmin(r))
    # refine with a parabola through the three best points
    w0 = ws[i]
    if 0 < i < len(ws) - 1:
        y0, y1, y2 = r[i - 1], r[i], r[i + 1]
        h = ws[1] - ws[0]
        w0 = ws[i] + 0.5 * h * (y0 - y2) / (y0 - 2 * y1 + y2)
    omega = w0 / wl.dt  # radians per unit time (omega_p = 1)
    expect = (2.0 / wl.dt) * math.asin(0.1 / 2.0)
    assert abs(expect - 1.000417) < 1e-6
    assert abs(omega / expect - 1.0) < 1e-4
    # the pin can tell leapfrog from the exact plasma frequency
    assert abs(omega - 1.0) > 2e-4
