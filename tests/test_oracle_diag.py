"""Pins of the oracle's diagnostics (the per-species count, kinetic energy and
momentum, and the field energy of the last solve; Sec. 2, the quantities a
PIC cycle reports), of its FP32 storage rounding and of the wall tie.

Closed forms used:
  * particles with a known SI velocity: KE = 1/2 m w N |V|^2 and momentum
    m w N V exactly (pins the cells/step -> m/s conversion and the 1/2);
  * a drawn Maxwellian at temperature T: KE = 3/2 N w T within its sampling
    error sqrt(2/(3N));
  * a uniform charge slab rho0 between grounded walls: the discrete field is
    the exact E = rho0 (2x - L) / (2 eps0) at every node (half-cell Gauss
    closure included), so the trapezoid energy 1/2 eps0 sum E_j^2 V_j (wall
    nodes V = dx/2) is rho0^2 L^3 (1 + 2/nc^2) / (24 eps0) exactly;
  * a periodic charge wave rho_j = rho1 cos(k x_j + c): the discrete
    eigenvector gives E_j = rho1 dx sin(k dx) / (eps0 lam) sin(k x_j + c) with
    lam = 4 sin^2(k dx / 2), energy 1/2 eps0 dx (amplitude)^2 nc/2;
  * a periodic plasma on an immobile background conserves the momentum of its
    mobile species (linear weights for both deposit and gather, central
    differences of a discrete Poisson solution: sum_j rho_j E_j = 0).
"""
import math

import numpy as np
import pytest

import pic_inputs as pin


def _empty(n_sp):
    return [pin.SpeciesState(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0),
                             id=np.zeros(0, np.uint64)) for _ in range(n_sp)]


def _beam_workload(nc=50, bc=pin.BC_PERIODIC):
    dx, dt = 2.5e-6, 4.0e-14
    e = pin.Species("e", pin.KIND_ELECTRON, q=-pin.E_CHARGE, m=pin.M_ELECTRON, w=3.0e13, ppc=0, T=0)
    i = pin.Species("i", pin.KIND_ION, q=pin.E_CHARGE, m=1836.0 * pin.M_ELECTRON, w=7.0e12,
                    ppc=0, T=0)
    return pin.Workload(name="beam", nc=nc, bc=bc, dx=dx, dt=dt, eps0=pin.EPS0_SI, species=[e, i])


def test_kinetic_energy_and_momentum_of_a_known_beam(oracle_lib):
    """Electrons at V = (3e5, -4e5, 1.2e6) m/s and ions at (-2e3, 5e3, 7e2) m/s:
    KE = 1/2 m w N |V|^2, momentum m w N V per component (component order kept)."""
    wl = _beam_workload()
    vs = wl.dt / wl.dx  # m/s -> cells per step
    V = [np.array([3e5, -4e5, 1.2e6]), np.array([-2e3, 5e3, 7e2])]
    N = [37, 11]
    st = []
    for k in range(2):
        n = N[k]
        st.append(pin.SpeciesState(x=np.linspace(0.5, wl.nc - 0.5, n), vx=np.full(n, V[k][0] * vs),
                                   vy=np.full(n, V[k][1] * vs), vz=np.full(n, V[k][2] * vs),
                                   id=np.arange(n, dtype=np.uint64) + 100 * k))
    o = oracle_lib.OracleSim(wl, st, caps=N)
    d = o.diagnostics()
    for k, s in enumerate(wl.species):
        assert d.n[k] == N[k]
        ke = 0.5 * s.m * s.w * N[k] * float(V[k] @ V[k])
        assert abs(d.ke[k] / ke - 1.0) <= 1e-13
        for c in range(3):
            p = s.m * s.w * N[k] * V[k][c]
            assert abs(d.mom[k][c] - p) <= 1e-13 * abs(p)


def test_kinetic_energy_of_the_drawn_maxwellian(oracle_lib):
    """The drawn initial state at T_e = T_i = 20 eV: KE_s = 3/2 N_s w_s T_s within
    five standard deviations of its sampling error (relative sqrt(2/(3N)))."""
    wl = pin.bounded_mcc(nc=1000, ppc=100, seed=5)
    st = oracle_lib.init_state(wl)
    o = oracle_lib.OracleSim(wl, st)
    d = o.diagnostics()
    for k, s in enumerate(wl.species):
        n = st[k].n
        expect = 1.5 * n * s.w * s.T
        sigma = math.sqrt(2.0 / (3.0 * n))
        assert abs(d.ke[k] / expect - 1.0) <= 5.0 * sigma, (k, d.ke[k] / expect - 1.0)
        # the mean momentum of a Maxwellian is zero within sqrt(m T / N) per particle
        for c in range(3):
            assert abs(d.mom[k][c]) <= 5.0 * s.w * math.sqrt(s.m * s.T * n)


@pytest.mark.parametrize("nc", [16, 101, 1000])
def test_field_energy_of_a_uniform_slab_between_grounded_walls(oracle_lib, nc):
    wl = _beam_workload(nc=nc, bc=pin.BC_ABSORB)
    o = oracle_lib.OracleSim(wl, _empty(2), caps=[1, 1])
    ppc = 8  # ions per cell; the wall nodes own half a cell and get half as much
    S = np.full(nc + 1, ppc << 32, dtype=np.uint64)
    S[0] = S[nc] = (ppc // 2) << 32
    o.S[1][:] = S
    o.field()
    s = wl.species[1]
    rho0 = s.q * s.w * ppc / wl.dx
    assert np.allclose(o.rho, rho0, rtol=1e-15, atol=0)
    L = nc * wl.dx
    x = np.arange(nc + 1) * wl.dx
    assert np.max(np.abs(o.E - rho0 * (2 * x - L) / (2 * wl.eps0))) <= 1e-12 * rho0 * L / wl.eps0
    fe = o.diagnostics().field_energy
    expect = rho0 ** 2 * L ** 3 * (1.0 + 2.0 / nc ** 2) / (24.0 * wl.eps0)
    assert abs(fe / expect - 1.0) <= 1e-11, fe / expect - 1.0


@pytest.mark.parametrize("nc,mode", [(64, 1), (64, 5), (250, 17)])
def test_field_energy_of_a_periodic_charge_wave(oracle_lib, nc, mode):
    wl = _beam_workload(nc=nc, bc=pin.BC_PERIODIC)
    wl.species[1].w = wl.species[0].w  # equal weights: the wave is neutral on average
    o = oracle_lib.OracleSim(wl, _empty(2), caps=[1, 1])
    A = 1000.0  # particles per node; the ions carry A (1 + cos), the electrons A
    k = 2 * math.pi * mode / (nc * wl.dx)
    ph = k * wl.dx * np.arange(nc + 1) + 0.3
    Si = np.rint(A * (1.0 + np.cos(ph)) * 2.0 ** 32).astype(np.uint64)
    Si[nc] = 0  # node nc is node 0; put its charge on node 0 only
    Se = np.full(nc + 1, int(A) << 32, dtype=np.uint64)
    Se[nc] = 0
    o.S[0][:] = Se
    o.S[1][:] = Si
    o.field()
    rho = o.rho[:nc]
    # the realised wave (integer rounding of the deposit) has amplitude rho1 and phase 0.3
    c = np.cos(ph[:nc])
    s_ = np.sin(ph[:nc])
    rho1 = 2.0 * float(rho @ c) / nc
    assert abs(2.0 * float(rho @ s_) / nc) <= 1e-6 * abs(rho1)
    lam = 4.0 * math.sin(k * wl.dx / 2) ** 2
    amp = rho1 * wl.dx * math.sin(k * wl.dx) / (wl.eps0 * lam)
    assert np.max(np.abs(o.E[:nc] - amp * s_)) <= 1e-6 * abs(amp)
    fe = o.diagnostics().field_energy
    expect = 0.5 * wl.eps0 * wl.dx * amp ** 2 * nc / 2.0
    assert abs(fe / expect - 1.0) <= 1e-6, fe / expect - 1.0


def test_periodic_plasma_conserves_momentum(oracle_lib):
    """Warm electrons with a density wave on an immobile background, 100 steps:
    the field exchanges momentum with the electrons every step, the total stays
    at its start to the rounding of the fixed-point deposit (2^-33 of a weight
    per particle) and of the sums."""
    wl = pin.langmuir(nc=64, ppc=50, perturb_amp=5e-2, seed=3)
    st = pin.initial_state(wl)
    o = oracle_lib.OracleSim(wl, st)
    p0 = np.array(o.diagnostics().mom[0][:])
    impulse = 0.0
    for _ in range(100):
        v0 = o.vx[0][:o.n(0)].copy()
        o.step(1)
        impulse += float(np.sum(np.abs(o.vx[0][:o.n(0)] - v0)))
    s = wl.species[0]
    vs = wl.dx / wl.dt
    p = np.array(o.diagnostics().mom[0][:])
    scale = s.m * s.w * vs * impulse  # sum of |momentum kicks| over all particles and steps
    assert scale > 0
    assert abs(p[0] - p0[0]) <= 1e-12 * scale, (p[0] - p0[0]) / scale
    # no force across x: vy, vz untouched (B = 0)
    assert p[1] == p0[1] and p[2] == p0[2]


def test_fp32_storage_form(oracle_lib):
    """cell = floor(x), f rounded to float; an f that rounds to 1 moves to offset 0
    of the next cell, or stays at the largest float below 1 in the last cell."""
    f = oracle_lib.fp32_form
    nc = 100
    assert f(5.25, nc) == 5.25
    assert f(0.0, nc) == 0.0
    assert f(3.0 + 1.0 / 3.0, nc) == 3.0 + float(np.float32(1.0 / 3.0))
    assert f(3.0 + 1.0 / 3.0, nc) == 3.0 + 0.3333333432674408
    assert f(7.0 + (1.0 - 2.0 ** -30), nc) == 8.0
    assert f(99.0 + (1.0 - 2.0 ** -30), nc) == 99.0 + (1.0 - 2.0 ** -24)
    # the largest value that still rounds below 1 keeps its cell
    assert f(7.0 + (1.0 - 2.0 ** -24), nc) == 7.0 + (1.0 - 2.0 ** -24)
    # against the workload module's own FP32 rounding, on random positions and on
    # offsets just below one
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.random(2000) * nc,
                        np.floor(rng.random(200) * nc) + (1.0 - rng.random(200) * 2.0 ** -25)])
    x = np.minimum(x, np.nextafter(float(nc), 0.0))
    ref = pin.to_fp32_form([pin.SpeciesState(x=x, vx=x, vy=x, vz=x, id=np.zeros(x.size, np.uint64))],
                           nc)[0].as_f64().x
    got = np.array([f(v, nc) for v in x])
    assert np.array_equal(got, ref)


def test_wall_tie_x_equal_nc_absorbed_x_equal_zero_kept(oracle_lib):
    """The domain is [0, nc): a particle landing exactly on x = nc leaves through
    the right wall, one landing exactly on x = 0 stays."""
    wl = _beam_workload(nc=20, bc=pin.BC_ABSORB)
    st = [pin.SpeciesState(x=np.array([19.5, 0.5, 10.0]), vx=np.array([0.5, -0.5, 0.0]),
                           vy=np.zeros(3), vz=np.zeros(3), id=np.arange(3, dtype=np.uint64)),
          _empty(1)[0]]
    o = oracle_lib.OracleSim(wl, st, caps=[3, 1])
    o.push()  # acc arrays are zero: no field
    o.walls()
    c = o.counters
    assert (c.absorbed[0][0], c.absorbed[0][1]) == (0, 1)
    s = o.state(0)
    assert sorted(s.id.tolist()) == [1, 2]
    assert s.x[s.id.tolist().index(1)] == 0.0
