"""Pins of the oracle's density smoother (Sec. 2, phase 2; binomial 1-2-1
filter on node charges, reflected at absorbing walls, wrapped when periodic):
the discrete transfer function cos^2(pi m / nc) of a periodic Fourier mode,
charge conservation, the unchanged constant, and the smoothing matrix written
out on a small grid."""
import math

import numpy as np
import pytest

import pic_inputs as pin


@pytest.mark.parametrize("m,passes", [(1, 1), (5, 1), (17, 3), (64, 2)])
def test_periodic_mode_transfer_function(oracle_lib, m, passes):
    nc = 128
    j = np.arange(nc + 1)
    rho = np.cos(2 * math.pi * m * j / nc) + 0.3 * np.sin(2 * math.pi * m * j / nc)
    V = np.ones(nc + 1)
    out = oracle_lib.smooth(rho, V, pin.BC_PERIODIC, passes)
    gain = math.cos(math.pi * m / nc) ** (2 * passes)
    assert np.max(np.abs(out - gain * rho)) <= 1e-13


@pytest.mark.parametrize("bc", [pin.BC_ABSORB, pin.BC_PERIODIC])
def test_charge_conserved_and_constant_kept(oracle_lib, bc):
    nc = 97
    rng = np.random.default_rng(3)
    rho = rng.normal(size=nc + 1)
    V = np.ones(nc + 1)
    if bc == pin.BC_ABSORB:
        V[0] = V[nc] = 0.5
    else:
        rho[nc] = rho[0]
    out = oracle_lib.smooth(rho, V, bc, 4)
    n = nc if bc == pin.BC_PERIODIC else nc + 1
    assert abs(np.sum(out[:n] * V[:n]) - np.sum(rho[:n] * V[:n])) <= 1e-12 * np.sum(np.abs(rho))
    const = np.full(nc + 1, 2.5)
    if bc == pin.BC_PERIODIC:
        assert np.max(np.abs(oracle_lib.smooth(const, V, bc, 3) - 2.5)) <= 1e-15
    else:
        # a uniform charge per node (Q_j = rho_j V_j constant) is a fixed point with walls
        q = 1.75 / V
        assert np.max(np.abs(oracle_lib.smooth(q, V, bc, 3) * V - 1.75)) <= 1e-15


def test_bounded_matches_the_matrix(oracle_lib):
    nc = 9
    n = nc + 1
    rng = np.random.default_rng(4)
    rho = rng.normal(size=n)
    V = np.ones(n)
    V[0] = V[-1] = 0.5
    # every node keeps 1/2 of its charge and gives 1/4 to each neighbour; the
    # quarter that would cross a wall stays on the wall node
    M = np.zeros((n, n))
    for i in range(n):
        M[i, i] += 0.5
        M[max(i - 1, 0), i] += 0.25
        M[min(i + 1, n - 1), i] += 0.25
    Q = rho * V
    for _ in range(2):
        Q = M @ Q
    ref = Q / V
    assert np.max(np.abs(oracle_lib.smooth(rho, V, pin.BC_ABSORB, 2) - ref)) <= 1e-14


def test_field_uses_the_smoothed_density(oracle_lib):
    """With the smoother on, the oracle's rho is the smoothed raw rho."""
    wl = pin.bounded(nc=64, ppc=20, seed=5, source=False)
    st = pin.initial_state(wl)
    st[1].x[:] = np.random.default_rng(6).random(st[1].n) * wl.nc  # break the neutral start
    raw = oracle_lib.OracleSim(wl, st)
    raw.deposit()
    raw.field()
    sm = oracle_lib.OracleSim(wl.replace(smooth_passes=2), st)
    sm.deposit()
    sm.field()
    V = np.full(wl.nc + 1, wl.dx)
    V[0] = V[-1] = 0.5 * wl.dx
    assert np.array_equal(sm.rho, oracle_lib.smooth(raw.rho, V, pin.BC_ABSORB, 2))
    assert not np.array_equal(sm.phi, raw.phi)
