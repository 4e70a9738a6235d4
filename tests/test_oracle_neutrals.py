"""Pins of the oracle's kinetic neutrals (the paper's Table 1 case, Sec. 3.4:
electrons, D+ ions and D atoms, no field solver, ionisation depleting the gas).

* the neutral decay law of Sec. 3.4 with the sign read as a loss,
  dn/dt = -n n_e R, for a constant rate coefficient R, whose solution with
  n_e = n_e0 + (n_0 - n) (each ionisation adds an electron) is logistic;
* every consumed atom becomes the new ion (same position and velocity) and
  lies in the parent electron's cell; the events of a cell take the atoms with
  the smallest keys; a cell short of atoms leaves events untargeted;
* excitation removes exactly E_ex and never acts below threshold; its count is
  the binomial expectation of the null-collision test;
* the node density of the neutrals is their linear-weight count times the
  macro weight over the node volume (numpy, independently);
* without the field solver every charged particle moves ballistically;
* the rate follows the local density: no event where no atom is near.
"""
import math

import numpy as np
import pytest

import oracle
import pic_inputs as pin


@pytest.fixture(scope="module", autouse=True)
def _lib(oracle_lib):
    return oracle_lib


def small(nc=100, ppc=100, ppc_n=None, L=1e-3, seed=31, **mcc_kw):
    """A Table 1 system of nc cells of 10 um (or L / nc) with its processes
    replaced by mcc_kw (others zero)."""
    base = dict(n_n=2e21, T_n=pin.EV, sig_el=0.0, sig_iz=0.0, E_iz=0.0, sig_cx=0.0,
                sig_ex=0.0, E_ex=0.0)
    base.update(mcc_kw)
    wl = pin.table1(nc=nc, ppc=ppc, L=L, seed=seed, mcc=pin.MCC(**base))
    if ppc_n is not None:
        n = wl.species[2]
        n.ppc = ppc_n
    return wl


def sim(wl, st):
    """The oracle with room for every atom to be ionised."""
    room = 2 * sum(x.n for x in st)
    return oracle.OracleSim(wl, st, caps=[room] * len(st))


def run_phases_to_mcc(o):
    """One step up to (not including) the collisions; returns the neutral,
    electron and ion states the collisions see."""
    o.deposit()
    o.field()
    o.push()
    o.walls()
    return [o.state(k) for k in range(3)]


def test_decay_law_constant_rate_coefficient():
    # R = sig_iz v_cap; every electron may ionise (no threshold); only ionisation
    wl = small(nc=100, ppc=100, ppc_n=200, sig_iz=1.0, E_iz=0.0, iz_const_rate=True, n_n=4e21)
    e = wl.species[0]
    # choose sig_iz so that nu_max dt = n_n sig v_cap dt = 2e-3
    sig = 2e-3 / (wl.mcc.n_n * e.v_cap * wl.dt)
    wl.mcc.sig_iz = sig
    st = pin.initial_state(wl)
    o = sim(wl, st)
    Ne0, N0 = st[0].n, st[2].n
    C = Ne0 + N0
    Lsys = wl.nc * wl.dx
    w = wl.species[2].w
    # per-step probability of the null-collision test: P = T 2^-32 over the
    # candidates, times the process share n_loc sig v_cap / nu_max = n_loc / n_n
    P = o.candidate_threshold(0) * 2.0 ** -32
    a = P * w / (Lsys * wl.mcc.n_n)      # events per step per (neutral, electron) pair
    checks = []
    for s_end in (100, 200, 300, 400):
        o.step(s_end - o.step_index)
        N = o.n(2)
        closed = C * N0 / (N0 + (C - N0) * math.exp(a * C * s_end))
        checks.append((s_end, N, closed))
        # the ledger: every ionisation consumed an atom, made an electron and an ion
        c = o.counters
        assert c.n_consumed == c.n_ionize and c.n_iz_untargeted == 0
        assert o.n(0) == Ne0 + (N0 - N) and o.n(1) == st[1].n + (N0 - N)
    assert (o.counters.status & oracle.ST_NN_CAP) == 0  # the bound held everywhere
    dep = N0 - checks[-1][1]
    assert dep > 0.2 * N0  # a real depletion
    for s_end, N, closed in checks:
        sigma = math.sqrt(max(N0 - closed, 1.0))
        assert abs(N - closed) < 5.0 * sigma + 1e-3 * N0, (s_end, N, closed)


def test_decay_is_faster_than_a_fixed_electron_count_would_give():
    """With n_e growing the logistic decay outruns the exponential one; the
    run separates the two (a sign or growth error in n_e would not)."""
    wl = small(nc=100, ppc=100, ppc_n=300, sig_iz=1.0, iz_const_rate=True, n_n=6e21)
    e = wl.species[0]
    wl.mcc.sig_iz = 4e-3 / (wl.mcc.n_n * e.v_cap * wl.dt)
    st = pin.initial_state(wl)
    o = sim(wl, st)
    Ne0, N0 = st[0].n, st[2].n
    P = o.candidate_threshold(0) * 2.0 ** -32
    a = P * wl.species[2].w / (wl.nc * wl.dx * wl.mcc.n_n)
    s = 300
    o.step(s)
    assert (o.counters.status & oracle.ST_NN_CAP) == 0
    N = o.n(2)
    expo = N0 * math.exp(-a * Ne0 * s)
    C = Ne0 + N0
    logi = C * N0 / (N0 + (C - N0) * math.exp(a * C * s))
    assert logi < expo - 10 * math.sqrt(N0 - logi)
    assert abs(N - logi) < 5 * math.sqrt(N0 - logi) + 1e-3 * N0


def _cells(x):
    return np.floor(x).astype(np.int64)


def test_consumed_atoms_become_the_ions_smallest_keys_first():
    # strong ionisation so that cells see several events in one step
    wl = small(nc=40, ppc=60, ppc_n=20, sig_iz=1.0, E_iz=0.0, iz_const_rate=True)
    e = wl.species[0]
    wl.mcc.sig_iz = 0.2 / (wl.mcc.n_n * e.v_cap * wl.dt)
    st = pin.initial_state(wl)
    o = sim(wl, st)
    o.step(1)
    step = o.step_index
    next_id = int(o.counters.next_id)
    before = run_phases_to_mcc(o)
    n0 = o.counters.n_consumed
    o.mcc()
    c = o.counters
    consumed = c.n_consumed - n0
    assert consumed > 30
    neu_b, neu_a = before[2], o.state(2)
    gone = np.setdiff1d(neu_b.id, neu_a.id)
    assert gone.size == consumed
    assert neu_a.n == neu_b.n - consumed
    idx_b = {int(i): q for q, i in enumerate(neu_b.id)}
    ions = o.state(1)
    elec = o.state(0)
    new_ion = ions.id >= next_id
    new_el = elec.id >= next_id
    el_by_id = {int(i): q for q, i in enumerate(elec.id)}
    # every consumed atom is exactly one new ion: same position and velocity
    atoms = {(neu_b.x[idx_b[int(g)]], neu_b.vx[idx_b[int(g)]], neu_b.vy[idx_b[int(g)]],
              neu_b.vz[idx_b[int(g)]]) for g in gone}
    ion_states = [(ions.x[q], ions.vx[q], ions.vy[q], ions.vz[q]) for q in np.flatnonzero(new_ion)]
    matched = [s for s in ion_states if s in atoms]
    assert len(matched) == consumed
    # ... in the cell of its event's parent (= the new electron of the pair)
    for q in np.flatnonzero(new_ion):
        pe = el_by_id[int(ions.id[q]) - 1]
        assert math.floor(elec.x[pe]) == math.floor(ions.x[q])
    # per cell: events (parent cells) take min(events, atoms) atoms with the smallest keys
    ev_cells = _cells(elec.x[new_el])
    cells_b = _cells(neu_b.x)
    gone_set = set(int(g) for g in gone)
    for j in np.unique(ev_cells):
        n_ev = int(np.sum(ev_cells == j))
        ids = neu_b.id[cells_b == j]
        keys = sorted((o.neutral_key(int(i), step), int(i)) for i in ids)
        want = {i for _, i in keys[:min(n_ev, len(keys))]}
        got = {int(i) for i in ids if int(i) in gone_set}
        assert got == want, j
    assert c.n_iz_untargeted >= 0


def test_cells_short_of_atoms_leave_events_untargeted():
    wl = small(nc=20, ppc=100, ppc_n=1, sig_iz=1.0, iz_const_rate=True, n_n=5e19)
    e = wl.species[0]
    wl.mcc.sig_iz = 0.5 / (wl.mcc.n_n * e.v_cap * wl.dt)
    st = pin.initial_state(wl)
    o = sim(wl, st)
    next_id = int(o.counters.next_id)
    before = run_phases_to_mcc(o)
    o.mcc()
    c = o.counters
    assert c.n_ionize > 0 and c.n_iz_untargeted > 0
    assert c.n_consumed + c.n_iz_untargeted == c.n_ionize
    elec = o.state(0)
    ev_cells = _cells(elec.x[elec.id >= next_id])
    cells_b = _cells(before[2].x)
    expect = sum(min(int(np.sum(ev_cells == j)), int(np.sum(cells_b == j)))
                 for j in np.unique(ev_cells))
    assert c.n_consumed == expect
    # untargeted ions sit at their parent with a fresh Maxwellian draw
    ions = o.state(1)
    assert int(np.sum(ions.id >= next_id)) == c.n_ionize


def test_excitation_energy_budget_and_threshold():
    E_ex = 20.0 * pin.EV
    wl = small(nc=50, ppc=400, sig_ex=1.0, E_ex=E_ex)
    e = wl.species[0]
    wl.mcc.sig_ex = 0.2 / (wl.mcc.n_n * e.v_cap * wl.dt)
    st = pin.initial_state(wl)
    o = sim(wl, st)
    before = run_phases_to_mcc(o)
    o.mcc()
    c = o.counters
    assert c.n_excite > 100 and c.n_ionize == 0 and c.n_elastic == 0
    eb, ea = before[0], o.state(0)
    assert np.array_equal(eb.id, ea.id)
    v2b = (eb.vx ** 2 + eb.vy ** 2) + eb.vz ** 2
    v2a = (ea.vx ** 2 + ea.vy ** 2) + ea.vz ** 2
    changed = (eb.vx != ea.vx) | (eb.vy != ea.vy) | (eb.vz != ea.vz)
    assert int(changed.sum()) == c.n_excite
    v2_ex = 2.0 * E_ex / e.m * (wl.dt / wl.dx) ** 2
    assert np.all(v2b[changed] >= v2_ex)
    np.testing.assert_allclose(v2a[changed], v2b[changed] - v2_ex, rtol=1e-12, atol=1e-12 * v2_ex)
    # count: the null-collision test gives P_cand * (n_loc sig_ex |v| / nu_max) per electron
    P = o.candidate_threshold(0) * 2.0 ** -32
    vcap = e.v_cap * wl.dt / wl.dx
    nloc = np.interp(eb.x, np.arange(wl.nc + 1), o.nn)
    p = P * (nloc / wl.mcc.n_n) * np.sqrt(v2b) / vcap * (v2b >= v2_ex)
    mu, var = p.sum(), (p * (1 - p)).sum()
    assert abs(c.n_excite - mu) < 5 * math.sqrt(var)


def test_neutral_density_is_the_weighted_count_over_the_node_volume():
    for bc in (pin.BC_PERIODIC, pin.BC_ABSORB):
        wl = small(nc=64, ppc=30, ppc_n=45).replace(bc=bc)
        st = pin.initial_state(wl)
        o = sim(wl, st)
        o.deposit()
        o.field()
        x = st[2].x
        j = np.floor(x).astype(np.int64)
        f = x - j
        cnt = np.zeros(wl.nc + 1)
        np.add.at(cnt, j, 1.0 - f)
        np.add.at(cnt, j + 1, f)
        V = np.full(wl.nc + 1, wl.dx)
        if bc == pin.BC_PERIODIC:
            cnt[0] += cnt[wl.nc]
            cnt[wl.nc] = cnt[0]
        else:
            V[0] = V[-1] = 0.5 * wl.dx
        ref = wl.species[2].w * cnt / V
        # the deposit rounds each weight to 2^-32
        np.testing.assert_allclose(o.nn, ref, rtol=1e-9)
        # total: integral of the density = real atoms per unit area
        vol = V.copy()
        if bc == pin.BC_PERIODIC:
            vol[-1] = 0.0
        assert math.isclose(float(np.sum(o.nn * vol)), wl.species[2].w * x.size, rel_tol=1e-12)


def test_without_the_field_solver_everything_moves_ballistically():
    wl = small(nc=32, ppc=20).replace(mcc=None)
    st = pin.initial_state(wl)
    o = sim(wl, st)
    o.step(7)
    o.deposit()
    o.field()
    assert np.all(o.E == 0.0) and np.all(o.phi == 0.0)
    assert all(np.all(a == 0.0) for a in o.acc)
    for k in range(3):
        s = o.state(k)
        order = np.argsort(s.id)
        s0 = st[k]
        np.testing.assert_array_equal(s.vx[order], s0.vx)
        np.testing.assert_array_equal(s.vz[order], s0.vz)
        x = s0.x.copy()
        for _ in range(7):
            x = x + s0.vx
            x = np.where(x < 0, x + wl.nc, x)
            x = np.where(x >= wl.nc, x - wl.nc, x)
        np.testing.assert_array_equal(s.x[order], x)
    # with the field solver the same plasma would be accelerated
    o2 = oracle.OracleSim(wl.replace(field_off=False), st)
    o2.deposit()
    o2.field()
    assert np.any(o2.E != 0.0)


def test_rate_follows_the_local_density():
    """Atoms only in the left half: ionisation happens only where the gathered
    density is positive, at the local (not the mean) rate."""
    wl = small(nc=100, ppc=200, ppc_n=100, sig_iz=1.0, iz_const_rate=True, n_n=4e21)
    e = wl.species[0]
    wl.mcc.sig_iz = 0.1 / (wl.mcc.n_n * e.v_cap * wl.dt)
    st = pin.initial_state(wl)
    st[2].x[:] = st[2].x * 0.5          # atoms in [0, nc/2)
    o = sim(wl, st)
    next_id = int(o.counters.next_id)
    before = run_phases_to_mcc(o)
    o.mcc()
    elec = o.state(0)
    xe = elec.x[elec.id >= next_id]
    assert xe.size > 50
    nloc = np.interp(xe, np.arange(wl.nc + 1), o.nn)
    assert np.all(nloc > 0)
    # no event between the atoms' last node (nc/2) and the periodic image of
    # node 0 (node nc)
    assert not np.any((xe >= 0.5 * wl.nc + 1) & (xe < wl.nc - 1))
    # rate: expected events from the local density of every electron
    eb = before[0]
    P = o.candidate_threshold(0) * 2.0 ** -32
    nl = np.interp(eb.x, np.arange(wl.nc + 1), o.nn)
    p = P * nl / wl.mcc.n_n
    mu, var = p.sum(), (p * (1 - p)).sum()
    assert abs(xe.size - mu) < 5 * math.sqrt(var)
