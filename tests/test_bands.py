"""Mean-free-path band discretisation (Sec. 3.1, eq. banddis).

Oracle pins (from the equation, not re-typed): the band sums conserve the
total heat capacity, sum C v and the bulk conductivity sum C v^2 tau; each
band's mean free path v_b tau_b lies within its modes' range; a band of one
mode is that mode; zero-speed modes add heat capacity only; permuting the
modes or scaling every tau changes nothing but tau (scaled).
Parity (host code, no GPU): bte_band_discretize through the C ABI against
the oracle on seeded synthetic mode lists -- band indices bit-exact (both
decide the interval with the same libm log in FP64), band values within
1e-13 relative (summation order is the same; contraction may differ).
"""
import ctypes as C

import numpy as np
import pytest

import bte_inputs as I
from oracle.bands import band_discretize as oracle_bands


def totals(Cm, vm, tm):
    Cm, vm, tm = (np.asarray(a, dtype=np.float64) for a in (Cm, vm, tm))
    return np.array([Cm.sum(), (Cm * vm).sum(), (Cm * vm * vm * tm).sum()])


@pytest.mark.parametrize("nb", [1, 7, 20, 40])
def test_oracle_conserves_band_sums(nb):
    m = I.modes(1, 3000)
    Cb, vb, tb, idx = oracle_bands(m["C"], m["v"], m["tau"], nb)
    assert 1 <= len(Cb) <= nb
    np.testing.assert_allclose(totals(Cb, vb, tb), totals(m["C"], m["v"], m["tau"]), rtol=1e-13)
    # ascending mean free path, each within the range of its own modes
    lam_b = np.array(vb) * np.array(tb)
    assert np.all(np.diff(lam_b) > 0)
    lam = m["v"] * m["tau"]
    idx = np.array(idx)
    for b in range(len(Cb)):
        sel = (idx == b) & (lam > 0)
        assert lam[sel].min() * (1 - 1e-14) <= lam_b[b] <= lam[sel].max() * (1 + 1e-14)


def test_oracle_single_mode_bands_are_the_modes():
    # mean free paths 1e-9, 3e-8, 3e-7, 1e-6 m in three decades: the first
    # two intervals hold one mode each, the last (closed) two
    Cm = np.array([2.0e5, 3.0e5, 4.0e5, 5.0e5])
    vm = np.array([1000.0, 3000.0, 3000.0, 5000.0])
    tm = np.array([1e-12, 1e-11, 1e-10, 2e-10])
    Cb, vb, tb, idx = oracle_bands(Cm, vm, tm, 3)
    assert idx == [0, 1, 2, 2]
    for b in (0, 1):
        assert (Cb[b], vb[b]) == (Cm[b], vm[b])
        assert abs(tb[b] - tm[b]) <= 1e-15 * tm[b]
    # the merged band: conductivity-preserving average of the two modes
    np.testing.assert_allclose(Cb[2] * vb[2] ** 2 * tb[2], (Cm[2:] * vm[2:] ** 2 * tm[2:]).sum(), rtol=1e-15)


def test_oracle_zero_speed_modes_only_add_heat_capacity():
    m = I.modes(2, 500, frac_zero_v=0.0)
    Cb, vb, tb, _ = oracle_bands(m["C"], m["v"], m["tau"], 10)
    Cz = np.concatenate([m["C"], [1e4, 2e4]])
    vz = np.concatenate([m["v"], [0.0, 0.0]])
    tz = np.concatenate([m["tau"], [1e-12, 1e-9]])
    Cb2, vb2, tb2, idx2 = oracle_bands(Cz, vz, tz, 10)
    assert idx2[-2:] == [0, 0]
    assert abs(Cb2[0] - (Cb[0] + 3e4)) <= 1e-12 * Cb2[0]
    np.testing.assert_allclose(np.array(Cb2[1:]), Cb[1:], rtol=0)
    # sum C v and sum C v^2 tau of band 0 are unchanged
    np.testing.assert_allclose(Cb2[0] * vb2[0], Cb[0] * vb[0], rtol=1e-14)
    np.testing.assert_allclose(Cb2[0] * vb2[0] ** 2 * tb2[0], Cb[0] * vb[0] ** 2 * tb[0], rtol=1e-14)


def test_oracle_permutation_and_tau_scaling():
    m = I.modes(3, 2000)
    Cb, vb, tb, _ = oracle_bands(m["C"], m["v"], m["tau"], 15)
    p = np.random.default_rng(0).permutation(2000)
    Cp, vp, tp, _ = oracle_bands(m["C"][p], m["v"][p], m["tau"][p], 15)
    np.testing.assert_allclose(Cp, Cb, rtol=1e-13)
    np.testing.assert_allclose(vp, vb, rtol=1e-13)
    np.testing.assert_allclose(tp, tb, rtol=1e-13)
    Cs, vs, ts, _ = oracle_bands(m["C"], m["v"], m["tau"] * 4.0, 15)   # a power of two: same bins exactly
    np.testing.assert_allclose(Cs, Cb, rtol=0)
    np.testing.assert_allclose(np.array(ts), 4.0 * np.array(tb), rtol=1e-15)


@pytest.fixture(scope="module")
def lib():
    from paper_2306_14181_amd import bte
    return bte


@pytest.mark.parametrize("n,nb", [(2000, 10), (100000, 20), (100000, 40), (50, 64)])
def test_abi_matches_oracle(lib, n, nb):
    m = I.modes(10 + nb, n)
    got, band = lib.band_discretize(m["C"], m["v"], m["tau"], nb)
    Cb, vb, tb, idx = oracle_bands(m["C"], m["v"], m["tau"], nb)
    assert np.array_equal(band, np.array(idx, dtype=np.int32))
    assert len(got["C"]) == len(Cb)
    np.testing.assert_allclose(got["C"], Cb, rtol=1e-13)
    np.testing.assert_allclose(got["v"], vb, rtol=1e-13)
    np.testing.assert_allclose(got["tau"], tb, rtol=1e-13)


@pytest.mark.parametrize("bad", ["no_positive_mfp", "negative_C", "zero_tau", "n_bands", "empty"])
def test_abi_rejects_invalid_lists(lib, bad):
    m = I.modes(4, 20)
    Cm, vm, tm, nb = m["C"].copy(), m["v"].copy(), m["tau"].copy(), 5
    if bad == "no_positive_mfp":
        vm[:] = 0.0
    elif bad == "negative_C":
        Cm[3] = -1.0
    elif bad == "zero_tau":
        tm[7] = 0.0
    elif bad == "n_bands":
        nb = 0
    else:
        Cm, vm, tm = Cm[:0], vm[:0], tm[:0]
    with pytest.raises(lib.BteError):
        lib.band_discretize(Cm, vm, tm, nb)


def test_bands_feed_a_problem(lib):
    """The discretised bands are a valid PHONON input (bte_setup accepts
    them) and keep the bulk conductivity of the mode list."""
    from tests.helpers import geo
    m = I.modes(5, 5000)
    bands, _ = lib.band_discretize(m["C"], m["v"], m["tau"], 12)
    k_modes = (m["C"] * m["v"] ** 2 * m["tau"]).sum() / 3
    k_bands = (bands["C"] * bands["v"] ** 2 * bands["tau"]).sum() / 3
    assert abs(k_bands - k_modes) <= 1e-13 * k_modes
    mat = dict(bands, n_theta=2, n_phi=2, Tref=300.0)
    g = geo(2, (4, 4), (1e-7, 1e-7), [I.BC_SPECULAR] * 6)
    from tests.test_abi import _setup
    st, h = _setup(lib.load(), g, mat)
    assert st == 0
    lib.load().bte_destroy(h)
