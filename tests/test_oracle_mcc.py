"""Pins of the oracle's Monte Carlo collision phase (Sec. 2, phase 4: Monte
Carlo collisions and ionisation), the pair source, created-particle ids and
resume.

The null-collision method is checked statistically against its defining
probabilities (binomial candidate and process counts), the collision
kinematics against conservation laws and the moments of isotropic scattering,
and the bookkeeping against exact ledgers.
"""
import math

import numpy as np
import pytest

import pic_inputs as pin


def _mcc_workload(nc=64, mass_ratio=1836.0, sig_el=1e-19, sig_iz=1e-21, sig_cx=5e-19,
                  source=False):
    wl = pin.bounded_mcc(nc=nc, ppc=1, mass_ratio=mass_ratio, source=source)
    mc = wl.mcc
    mc.sig_el, mc.sig_iz, mc.sig_cx = sig_el, sig_iz, sig_cx
    return wl


def _beam(wl, n_e, n_i, ve, vi, seed=0):
    rng = np.random.default_rng(seed)
    nc = wl.nc
    st = []
    nid = 0
    for n, v in ((n_e, ve), (n_i, vi)):
        x = rng.random(n) * nc
        st.append(pin.SpeciesState(x=x, vx=np.full(n, v[0]), vy=np.full(n, v[1]),
                                   vz=np.full(n, v[2]), id=np.arange(nid, nid + n, dtype=np.uint64)))
        nid += n
    return st


def _speed_hat_for_energy(wl, k, E_eV):
    s = wl.species[k]
    v = math.sqrt(2.0 * E_eV * pin.EV / s.m)
    return v * wl.dt / wl.dx


def _zscore(k, n, p):
    return (k - n * p) / math.sqrt(n * p * (1 - p))


def test_candidate_and_elastic_counts_binomial(oracle_lib):
    wl = _mcc_workload()
    g = _speed_hat_for_energy(wl, 0, 10.0)  # below the 15 eV threshold: elastic only
    N = 400_000
    st = _beam(wl, N, 0, (g, 0.0, 0.0), (0, 0, 0))
    o = oracle_lib.OracleSim(wl, st, caps=[N + 10, 10])
    T = o.candidate_threshold(0)
    o.mcc()
    c = o.counters
    p = T / 2.0 ** 32
    assert abs(_zscore(c.n_candidates, N, p)) < 5
    # process choice: elastic with probability n_n sigma_el dx |v| / nu_max
    vcap = wl.species[0].v_cap * wl.dt / wl.dx
    p_el = (wl.mcc.sig_el * g) / ((wl.mcc.sig_el + wl.mcc.sig_iz) * vcap)
    assert abs(_zscore(c.n_elastic, c.n_candidates, p_el)) < 5
    assert c.n_ionize == 0
    # null collision reproduces the direct probability 1 - exp(-nu dt) to O((nu_max dt)^2)
    nu_el = wl.mcc.n_n * wl.mcc.sig_el * wl.dx * g
    direct = -math.expm1(-nu_el)
    nu_max = wl.mcc.n_n * (wl.mcc.sig_el + wl.mcc.sig_iz) * wl.dx * vcap
    assert abs(c.n_elastic / N - direct) < 5 * math.sqrt(direct / N) + nu_max ** 2


def test_candidate_threshold_probability(oracle_lib):
    """T / 2^32 = 1 - exp(-nu_max dt) for the electron and the ion species."""
    wl = _mcc_workload()
    st = _beam(wl, 1, 1, (0, 0, 0), (0, 0, 0))
    o = oracle_lib.OracleSim(wl, st)
    for k, sig in ((0, wl.mcc.sig_el + wl.mcc.sig_iz), (1, wl.mcc.sig_cx)):
        vcap = wl.species[k].v_cap  # m/s
        nu_max_dt = wl.mcc.n_n * sig * vcap * wl.dt  # physical rate times dt
        P = 1.0 - math.exp(-nu_max_dt)
        assert 0 <= P - o.candidate_threshold(k) / 2.0 ** 32 < 2.0 ** -32 + 1e-15  # floor
    # the defaults give the fractions quoted for the collisional workload
    assert abs(o.candidate_threshold(0) / 2.0 ** 32 - 0.0464) < 5e-4
    assert abs(o.candidate_threshold(1) / 2.0 ** 32 - 0.00548) < 5e-5


def test_elastic_kinematics_moments(oracle_lib):
    """Cold target of mass M, isotropic in the centre of mass:
    <v'> = m/(m+M) v and <|v'|^2>/|v|^2 = 1 - 2 m M/(m+M)^2."""
    wl = _mcc_workload(mass_ratio=4.0, sig_iz=0.0)
    g = _speed_hat_for_energy(wl, 0, 5.0)
    N = 1_000_000
    v0 = np.array([0.6, -0.48, 0.64]) * g  # |v0| = g
    st = _beam(wl, N, 0, tuple(v0), (0, 0, 0))
    o = oracle_lib.OracleSim(wl, st, caps=[N + 10, 10])
    o.mcc()
    s = o.state(0)
    v = np.stack([s.vx, s.vy, s.vz], 1)
    hit = np.any(v != v0[None, :], axis=1)
    n_hit = int(hit.sum())
    assert n_hit == o.counters.n_elastic and n_hit > 5000
    vh = v[hit]
    m, M = 1.0, 4.0
    a, b = m / (m + M), M / (m + M)
    mean = vh.mean(0)
    se = b * g / math.sqrt(3 * n_hit)
    assert np.all(np.abs(mean - a * v0) < 6 * se)
    e_ratio = np.sum(vh * vh, 1) / (g * g)
    expect = 1.0 - 2.0 * m * M / (m + M) ** 2
    se_e = 2 * a * b / math.sqrt(3 * n_hit)
    assert abs(e_ratio.mean() - expect) < 6 * se_e
    # the deflection (cos of the centre-of-mass angle) averages to zero:
    # R = (v' - a v)/(b g) is a unit vector uniform on the sphere
    R = (vh - a * v0[None, :]) / (b * g)
    assert np.allclose(np.linalg.norm(R, axis=1), 1.0, atol=1e-12)
    cos_chi = R @ (v0 / g)
    assert abs(cos_chi.mean()) < 6 / math.sqrt(3 * n_hit)


def test_ionisation_energy_budget_ids_and_positions(oracle_lib):
    wl = _mcc_workload(sig_el=0.0, sig_iz=1e-19)  # ionisation only
    g = _speed_hat_for_energy(wl, 0, 60.0)
    N = 100_000
    v0 = np.array([0.0, g, 0.0])
    st = _beam(wl, N, 5, tuple(v0), (0, 0, 0))
    o = oracle_lib.OracleSim(wl, st, caps=[2 * N, 2 * N])
    nid0 = int(o.sim.cnt.next_id)
    o.mcc()
    c = o.counters
    m_ev = c.n_ionize
    assert m_ev > 500
    s = o.state(0)
    old = s.id < nid0
    v = np.stack([s.vx, s.vy, s.vz], 1)
    changed = old & np.any(v != v0[None, :], axis=1)
    parents = np.sort(s.id[changed])
    assert parents.size == m_ev
    # new electrons: ids next_id0 + 2r in parent-id order
    new_e = ~old
    ids_e = s.id[new_e]
    order = np.argsort(ids_e)
    assert np.array_equal(ids_e[order], nid0 + 2 * np.arange(m_ev, dtype=np.uint64))
    si = o.state(1)
    new_i = si.id >= nid0
    ids_i = si.id[new_i]
    oi = np.argsort(ids_i)
    assert np.array_equal(ids_i[oi], nid0 + 2 * np.arange(m_ev, dtype=np.uint64) + 1)
    assert int(c.next_id) == nid0 + 2 * m_ev
    # energy: 1/2 |v1'|^2 + 1/2 |v2|^2 = 1/2 |v|^2 - eps_iz  (per unit mass, cells/step)
    eps_iz = wl.mcc.E_iz / wl.species[0].m * (wl.dt / wl.dx) ** 2
    par_idx = {int(i): n for n, i in enumerate(s.id)}
    e_prim = np.array([0.5 * np.sum(v[par_idx[int(p)]] ** 2) for p in parents])
    ve_new = v[new_e][order]
    e_sec = 0.5 * np.sum(ve_new ** 2, 1)
    lhs = e_prim + e_sec
    rhs = 0.5 * g * g - eps_iz
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * rhs
    # the pair is born at the parent's position
    xpar = np.array([s.x[par_idx[int(p)]] for p in parents])
    assert np.array_equal(s.x[new_e][order], xpar)
    assert np.array_equal(si.x[new_i][oi], xpar)
    # the new ion takes a neutral's Maxwellian velocity at T_n
    sig_i = math.sqrt(wl.mcc.T_n / wl.species[1].m) * wl.dt / wl.dx
    vi = np.stack([si.vx[new_i], si.vy[new_i], si.vz[new_i]], 1)
    assert abs(vi.std() / sig_i - 1.0) < 6 / math.sqrt(2 * vi.size)


def test_below_threshold_never_ionises(oracle_lib):
    wl = _mcc_workload(sig_el=0.0, sig_iz=1e-19)
    g = _speed_hat_for_energy(wl, 0, 14.9)
    st = _beam(wl, 50_000, 0, (g, 0.0, 0.0), (0, 0, 0))
    o = oracle_lib.OracleSim(wl, st)
    o.mcc()
    assert o.counters.n_candidates > 0 and o.counters.n_ionize == 0


def test_charge_exchange_maxwellian(oracle_lib):
    wl = _mcc_workload()
    g = _speed_hat_for_energy(wl, 1, 100.0)
    N = 300_000
    v0 = np.array([g, 0.0, 0.0])
    st = _beam(wl, 0, N, (0, 0, 0), tuple(v0))
    o = oracle_lib.OracleSim(wl, st, caps=[10, N + 10])
    o.mcc()
    s = o.state(1)
    v = np.stack([s.vx, s.vy, s.vz], 1)
    hit = np.any(v != v0[None, :], axis=1)
    n = int(hit.sum())
    assert n == o.counters.n_cx and n > 500
    sig_n = math.sqrt(wl.mcc.T_n / wl.species[1].m) * wl.dt / wl.dx
    vh = v[hit] / sig_n
    assert np.all(np.abs(vh.mean(0)) < 6 / math.sqrt(n))
    assert np.all(np.abs(vh.var(0) - 1.0) < 6 * math.sqrt(2.0 / n))


def test_source_pairs_uniform_and_maxwellian(oracle_lib):
    wl = _mcc_workload(source=True)
    wl.mcc = None
    st = _beam(wl, 0, 0, (0, 0, 0), (0, 0, 0))
    n_pairs = 20000
    o = oracle_lib.OracleSim(wl, st, caps=[n_pairs, n_pairs])
    o.sim.cnt.absorbed[1][0] = n_pairs - 7
    o.sim.cnt.absorbed[1][1] = 7
    o.sim.cnt.absorbed[0][0] = 12345  # electron losses do not drive the source
    o.source()
    se, si = o.state(0), o.state(1)
    assert se.n == n_pairs and si.n == n_pairs
    assert np.array_equal(se.id, 2 * np.arange(n_pairs, dtype=np.uint64))
    assert np.array_equal(si.id, 2 * np.arange(n_pairs, dtype=np.uint64) + 1)
    assert np.array_equal(se.x, si.x)
    assert np.all((se.x >= 0) & (se.x < wl.nc))
    # Kolmogorov-Smirnov against uniform [0, nc)
    u = np.sort(se.x / wl.nc)
    D = np.max(np.maximum(np.arange(1, u.size + 1) / u.size - u, u - np.arange(u.size) / u.size))
    assert D < 1.63 / math.sqrt(u.size)  # 1% level
    for k, s in ((0, se), (1, si)):
        sig = math.sqrt(wl.species[k].T_src / wl.species[k].m) * wl.dt / wl.dx
        v = np.stack([s.vx, s.vy, s.vz], 1) / sig
        assert np.all(np.abs(v.mean(0)) < 6 / math.sqrt(n_pairs))
        assert np.all(np.abs(v.var(0) - 1) < 6 * math.sqrt(2.0 / n_pairs))


@pytest.fixture(scope="module")
def mcc_run(oracle_lib):
    wl = pin.bounded_mcc(nc=256, ppc=40, n_steps=60)
    st = pin.initial_state(wl)
    return wl, st


def test_particle_ledger_and_unique_ids(oracle_lib, mcc_run):
    wl, st = mcc_run
    o = oracle_lib.OracleSim(wl, st)
    for _ in range(wl.n_steps):
        n_before = [o.n(0), o.n(1)]
        created_before = [int(o.counters.created_total[0]), int(o.counters.created_total[1])]
        nid_before = int(o.counters.next_id)
        o.step(1)
        c = o.counters
        for k in range(2):
            absorbed = int(c.absorbed[k][0] + c.absorbed[k][1])
            created = int(c.created_total[k]) - created_before[k]
            assert o.n(k) == n_before[k] - absorbed + created
        # every created particle consumed one id; electrons even offsets, ions odd
        assert int(c.next_id) - nid_before == (int(c.created_total[0]) - created_before[0]
                                               + int(c.created_total[1]) - created_before[1])
        ids = np.concatenate([o.state(0).id, o.state(1).id])
        assert np.unique(ids).size == ids.size
    assert o.counters.n_ionize > 0 and o.counters.n_source > 0 and o.counters.status == 0


def test_resume_is_bit_identical(oracle_lib, mcc_run):
    wl, st = mcc_run
    a = oracle_lib.OracleSim(wl, st)
    a.step(30)
    b = oracle_lib.OracleSim(wl, st)
    b.step(15)
    snap = b.snapshot()
    b2 = oracle_lib.OracleSim.from_snapshot(wl, snap)
    b2.step(15)
    for k in range(2):
        sa, sb = a.state(k), b2.state(k)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(getattr(sa, f), getattr(sb, f))


def test_result_independent_of_particle_order(oracle_lib, mcc_run):
    """Draws are keyed by (id, step), so a permuted start gives the same particles."""
    wl, st = mcc_run
    rng = np.random.default_rng(9)
    st2 = []
    for s in st:
        p = rng.permutation(s.n)
        st2.append(pin.SpeciesState(x=s.x[p], vx=s.vx[p], vy=s.vy[p], vz=s.vz[p], id=s.id[p]))
    a = oracle_lib.OracleSim(wl, st)
    b = oracle_lib.OracleSim(wl, st2)
    a.step(20)
    b.step(20)
    for k in range(2):
        sa, sb = a.state(k), b.state(k)
        ia, ib = np.argsort(sa.id), np.argsort(sb.id)
        for f in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(getattr(sa, f)[ia], getattr(sb, f)[ib])
