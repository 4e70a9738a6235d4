"""Pins of the oracle's Poisson/field phase (Sec. 2, phase 3: a tridiagonal
solve of the 1D Poisson equation, then E = -grad(phi)).

The pins are independent of the oracle's own formulas: a dense LU solve from
numpy, the discrete sine/cosine eigenvectors of the second-difference
operator (closed forms), the Green's function of the Dirichlet operator
summed in extended precision, Gauss's law over the whole bounded domain,
and the zero-mean field of a periodic system.
"""
import math

import numpy as np
import pytest

import pic_inputs as pin


@pytest.mark.parametrize("n", [1, 2, 5, 33, 64])
def test_thomas_matches_dense_lu(oracle_lib, n):
    rng = np.random.default_rng(n)
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = np.abs(a) + np.abs(c) + rng.uniform(0.5, 2.0, n)
    d = rng.normal(size=n)
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    ref = np.linalg.solve(A, d)
    got = oracle_lib.thomas(a, b, c, d)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [3, 31, 63])
def test_thomas_laplacian_matches_dense_lu(oracle_lib, n):
    rng = np.random.default_rng(100 + n)
    a = np.ones(n); b = -2.0 * np.ones(n); c = np.ones(n)
    d = rng.normal(size=n)
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    ref = np.linalg.solve(A, d)
    got = oracle_lib.thomas(a, b, c, d)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)) * n


@pytest.mark.parametrize("n", [1, 2, 5, 33, 64])
def test_poisson_dirichlet_matches_dense_lu(oracle_lib, n):
    rng = np.random.default_rng(200 + n)
    d = rng.normal(size=n)
    A = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    ref = np.linalg.solve(A, d)
    got = oracle_lib.poisson_dirichlet(d)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)) * n


def _green_extended(d):
    """x_j = -[(n+1-j) sum_{i<=j} i d_i + j sum_{i>j} (n+1-i) d_i] / (n+1): the
    Green's function of tridiag(1, -2, 1) with x_0 = x_{n+1} = 0, summed in
    80-bit extended precision."""
    n = d.shape[0]
    L = np.longdouble
    i = np.arange(1, n + 1, dtype=L)
    dl = d.astype(L)
    lower = np.cumsum(i * dl)
    upper = np.cumsum(((n + 1 - i) * dl)[::-1])[::-1]
    upper = np.concatenate([upper[1:], [L(0)]])
    return (-((n + 1 - i) * lower + i * upper) / (n + 1)).astype(np.float64)


@pytest.mark.parametrize("n", [30_000, 300_000])
def test_poisson_dirichlet_large_n_against_extended_precision(oracle_lib, n):
    """White-noise charge on up to 3e5 nodes (a random-walk potential, the hard case
    for rounding): the solve stays within n eps max|x| of the exact solution.  A
    pivot recurrence den_u = -2 - c'_(u-1) misses this bound by 20x at 3e4 nodes
    and 190x at 3e5."""
    if np.finfo(np.longdouble).eps > 1e-18:
        pytest.skip("no 80-bit extended precision on this host")
    d = np.random.default_rng(7).normal(size=n)
    ref = _green_extended(d)
    got = oracle_lib.poisson_dirichlet(d)
    assert np.max(np.abs(got - ref)) <= n * 2.0 ** -52 * np.max(np.abs(ref))


def _sim_with_S(oracle_lib, wl, S_list):
    st = [pin.SpeciesState(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0),
                           id=np.zeros(0, dtype=np.uint64)) for _ in wl.species]
    o = oracle_lib.OracleSim(wl, st, caps=[1] * len(wl.species))
    for k, S in enumerate(S_list):
        o.S[k][:] = S
    return o


def _two_species_workload(nc, bc):
    # unit charges and weights, eps0 = 1, dx = 1: rho_j = (S+_j - S-_j) 2^-32 / V_j
    sp = [pin.Species("p", pin.KIND_ION, q=1.0, m=1.0, w=1.0, ppc=0, T=0),
          pin.Species("m", pin.KIND_ELECTRON, q=-1.0, m=1.0, w=1.0, ppc=0, T=0)]
    return pin.Workload(name="t", nc=nc, bc=bc, dx=1.0, dt=1.0, eps0=1.0, species=sp)


@pytest.mark.parametrize("m", [1, 3, 17])
def test_dirichlet_sine_mode_closed_form(oracle_lib, m):
    nc = 128
    wl = _two_species_workload(nc, pin.BC_ABSORB)
    j = np.arange(nc + 1)
    k = m * math.pi / nc
    A = 1000.0
    # rho_j = A sin(k j) on interior nodes (zero at both walls)
    Sp = np.round((A * (1.0 + 0.5 * np.sin(k * j))) * 2.0 ** 32).astype(np.uint64)
    Sm = np.round((A * 1.0) * 2.0 ** 32 * np.ones(nc + 1)).astype(np.uint64)
    o = _sim_with_S(oracle_lib, wl, [Sp, Sm])
    o.field()
    rho_target = 0.5 * A * np.sin(k * j)
    # discrete eigen-relation: phi_j = rho_j dx^2 / (eps0 4 sin^2(k/2))
    phi_ref = rho_target / (4.0 * math.sin(k / 2) ** 2)
    assert abs(o.phi[0]) == 0 and abs(o.phi[nc]) == 0
    scale = np.max(np.abs(phi_ref))
    assert np.max(np.abs(o.phi - phi_ref)) <= 1e-8 * scale
    # E = -dphi/dx at interior nodes: the central difference of a sine
    E_ref = -(phi_ref[2:] - phi_ref[:-2]) / 2.0
    assert np.max(np.abs(o.E[1:nc] - E_ref)) <= 1e-8 * scale


def test_gauss_identity_bounded(oracle_lib):
    """E_nc - E_0 = Q_total / eps0 with half-cell wall nodes."""
    nc = 300
    wl = _two_species_workload(nc, pin.BC_ABSORB)
    rng = np.random.default_rng(3)
    Sp = rng.integers(0, 2 ** 40, nc + 1, dtype=np.uint64)
    Sm = rng.integers(0, 2 ** 40, nc + 1, dtype=np.uint64)
    o = _sim_with_S(oracle_lib, wl, [Sp, Sm])
    o.field()
    V = np.ones(nc + 1); V[0] = V[nc] = 0.5
    Q = np.sum((Sp.astype(np.float64) - Sm.astype(np.float64)) * 2.0 ** -32)
    # the wall nodes' deposits are divided by V = 1/2 inside the oracle; Q is the raw charge
    assert abs((o.E[nc] - o.E[0]) - Q) <= 1e-9 * max(1.0, np.sum(np.abs(o.rho * V)))


@pytest.mark.parametrize("m", [1, 5])
def test_periodic_cosine_mode_and_zero_mean(oracle_lib, m):
    nc = 256
    wl = _two_species_workload(nc, pin.BC_PERIODIC)
    j = np.arange(nc + 1)
    k = 2 * math.pi * m / nc
    A = 500.0
    Sp = np.round(A * (1.0 + 0.5 * np.cos(k * j)) * 2.0 ** 32).astype(np.uint64)
    Sp[nc] = 0  # node nc is node 0
    Sm = np.round(A * 2.0 ** 32 * np.ones(nc + 1)).astype(np.uint64)
    Sm[nc] = 0
    o = _sim_with_S(oracle_lib, wl, [Sp, Sm])
    # neutral on its own: no background needed (both species have N = 0 particles)
    o.field()
    phi_ref = 0.5 * A * np.cos(k * j) / (4.0 * math.sin(k / 2) ** 2)
    # gauge phi_0 = 0
    phi_ref = phi_ref - phi_ref[0]
    scale = np.max(np.abs(phi_ref))
    assert np.max(np.abs(o.phi[:nc] - phi_ref[:nc])) <= 1e-7 * scale
    assert abs(np.sum(o.E[:nc])) <= 1e-9 * np.sum(np.abs(o.E[:nc]))
    assert o.E[nc] == o.E[0]


def test_periodic_background_neutralises(oracle_lib):
    """One electron species on a uniform background: sum rho = 0 and sum E = 0."""
    wl = pin.langmuir(nc=64, ppc=10)
    st = pin.initial_state(wl)
    o = oracle_lib.OracleSim(wl, st)
    o.deposit()
    o.field()
    assert abs(np.sum(o.rho[:64])) <= 1e-10 * np.sum(np.abs(o.rho[:64]))
    assert abs(np.sum(o.E[:64])) <= 1e-10 * np.sum(np.abs(o.E[:64]))


def test_uniform_charge_parabola(oracle_lib):
    """Uniform rho between grounded walls: phi = rho x (L - x) / (2 eps0), exactly quadratic."""
    nc = 50
    wl = _two_species_workload(nc, pin.BC_ABSORB)
    Sp = np.full(nc + 1, 3 * 2 ** 32, dtype=np.uint64)
    Sp[0] = Sp[nc] = 3 * 2 ** 31  # half cells at the walls -> uniform density
    Sm = np.zeros(nc + 1, dtype=np.uint64)
    o = _sim_with_S(oracle_lib, wl, [Sp, Sm])
    o.field()
    x = np.arange(nc + 1, dtype=np.float64)
    phi_ref = 3.0 * x * (nc - x) / 2.0
    assert np.allclose(o.rho, 3.0, rtol=0, atol=1e-12)
    assert np.max(np.abs(o.phi - phi_ref)) <= 1e-10 * np.max(phi_ref)
    # E = -dphi/dx = -3 (L/2 - x) : linear, and the wall closure continues it exactly
    assert np.max(np.abs(o.E - (-3.0 * (nc / 2.0 - x)))) <= 1e-9 * nc
