"""Pins of the oracle's generator-drawn initial state (orc_init_species):
uniform positions (Kolmogorov-Smirnov), Maxwellian velocities (moments and
KS against the normal law), exact lattice and pair positions, the mode-1
density perturbation of the Langmuir start (X28), ids, and independence of
instances."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import pic_inputs as pin


@pytest.fixture(scope="module", autouse=True)
def _lib(oracle_lib):
    return oracle_lib


def test_counts_and_ids():
    wl = pin.bounded_mcc(nc=300, ppc=37.3)
    st = oracle.init_state(wl)
    n = int(round(37.3 * 300))
    assert [s.n for s in st] == [n, n]
    assert np.array_equal(st[0].id, np.arange(n, dtype=np.uint64))
    assert np.array_equal(st[1].id, np.arange(n, 2 * n, dtype=np.uint64))


def test_positions_uniform_and_inside():
    wl = pin.bounded_mcc(nc=1000, ppc=60, seed=21)
    st = oracle.init_state(wl)
    x = st[0].x
    assert np.all((x >= 0) & (x < wl.nc))
    assert stats.kstest(x / wl.nc, "uniform").pvalue > 1e-3


def test_velocities_maxwellian():
    wl = pin.bounded_mcc(nc=1000, ppc=60, seed=22)
    st = oracle.init_state(wl)
    for k, s in enumerate(wl.species):
        vth = wl.vth_hat(s)
        n = st[k].n
        for v in (st[k].vx, st[k].vy, st[k].vz):
            assert abs(v.mean()) < 5 * vth / math.sqrt(n)
            # variance of the sample variance of a normal: 2 vth^4 / n
            assert abs(v.var() - vth ** 2) < 5 * vth ** 2 * math.sqrt(2.0 / n)
            assert stats.kstest(v / vth, "norm").pvalue > 1e-3
        # components uncorrelated
        c = np.corrcoef([st[k].vx, st[k].vy, st[k].vz])
        assert np.max(np.abs(c - np.eye(3))) < 5 / math.sqrt(n)


def test_pair_start_copies_positions_only():
    wl = pin.bounded_mcc(nc=500, ppc=40, seed=23)
    assert wl.pair_start
    st = oracle.init_state(wl)
    assert np.array_equal(st[0].x, st[1].x)
    assert not np.array_equal(st[0].vx / wl.vth_hat(wl.species[0]),
                              st[1].vx / wl.vth_hat(wl.species[1]))
    wl2 = wl.replace(pair_start=False)
    st2 = oracle.init_state(wl2)
    assert np.array_equal(st2[0].x, st[0].x)
    assert stats.ks_2samp(st2[0].x, st2[1].x).pvalue > 1e-3
    assert np.mean(st2[0].x == st2[1].x) < 1e-3


def test_quiet_lattice_exact():
    wl = pin.langmuir(nc=64, ppc=10, quiet=True, perturb_amp=0.0)
    st = oracle.init_state(wl)
    n = 640
    assert np.array_equal(st[0].x, (np.arange(n) + 0.5) * 64 / n)
    assert np.all(st[0].vx == 0.0)  # cold


def test_mode1_perturbation_amplitude():
    """Displacement (A/k) sin(k x0) gives the density modulation -A cos(k x0)."""
    A = 1e-2
    wl = pin.langmuir(nc=256, ppc=200, quiet=True, perturb_amp=A)
    x = oracle.init_state(wl)[0].x
    k = 2 * math.pi / wl.nc
    # Fourier coefficient of the particle density in mode 1
    c1 = np.sum(np.exp(-1j * k * x)) / x.size
    assert abs(abs(c1) - A / 2) < 1e-3 * A
    # phase: density minimum where cos(k x0) = 1, i.e. coefficient real and negative
    assert c1.real < 0 and abs(c1.imag) < 1e-3 * A


def test_instances_draw_independently():
    wl = pin.bounded_mcc(nc=400, ppc=30, seed=24)
    a = oracle.init_state(wl, inst=0)
    b = oracle.init_state(wl, inst=1)
    assert np.mean(a[0].x == b[0].x) < 1e-3
    assert stats.ks_2samp(a[0].x, b[0].x).pvalue > 1e-3
