"""Pins of the oracle's colour shift for light of any colour (Section 3.4.2, the C(xy, D)
table; oracle/spectrum.c), against what the physics and the readings fix, computed here
with scipy quadrature of a Planck function written from its definition:

* the blackbody limit: D^5 B_T(D lambda) = B_{DT}(lambda), so a blackbody colour shifts
  to the band radiances of the blackbody at D T (per unit emitted band sum);
* at D = 1 the received colour is the emitted one (the chosen spectrum has the requested
  chromaticity), checked by integrating that spectrum independently;
* the correlated temperature has the requested blue-to-red ratio, and blackbody colours
  get their own temperature with no absorption;
* the absorption spectra, the clamps and the projection are as the readings state;
* the table holds the exact values at its nodes and interpolates as stated between them,
  and its distance to the exact shift is bounded on the colours the inputs use."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle

H, C, K = 6.62607015e-34, 299792458.0, 1.380649e-23
BANDS = ((600e-9, 700e-9), (500e-9, 600e-9), (400e-9, 500e-9))   # R, G, B


def planck(lam, T):
    return 2.0 * H * C * C / lam ** 5 / math.expm1(H * C / (lam * K * T))


def gauss(lam, mu):
    return math.exp(-0.5 * ((lam - mu) / 30e-9) ** 2)


def bands_of(f):
    return np.array([integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=200)[0]
                     for a, b in BANDS])


def bb_chroma(T):
    L = bands_of(lambda l: planck(l, T))
    return L / L.sum()


def in_gamut_grid():
    out = []
    for r in np.linspace(0.15, 0.55, 5):
        for g in np.linspace(0.2, 0.45, 5):
            if r + g < 0.9:
                T, a1, a2 = oracle.spectrum_of(r, g)
                if -8.0 < a1 < 1.0 and -8.0 < a2 < 1.0:
                    out.append((float(r), float(g)))
    return out


def test_absorption_spectra():
    assert oracle.absorption(0, 450e-9) == 1.0 and oracle.absorption(1, 650e-9) == 1.0
    assert oracle.absorption(0, 480e-9) == pytest.approx(math.exp(-0.5), rel=1e-14)
    assert oracle.absorption(1, 620e-9) == pytest.approx(math.exp(-0.5), rel=1e-14)
    lam = np.linspace(100e-9, 5000e-9, 4001)
    s = np.array([oracle.absorption(0, l) + oracle.absorption(1, l) for l in lam])
    assert s.max() <= 1.0 + 1e-9


def test_projection_onto_the_triangle():
    assert oracle.chroma_project(-0.1, 0.5) == (0.0, 0.5)
    r, g = oracle.chroma_project(0.8, 0.6)
    assert r == pytest.approx(0.8 / 1.4) and g == pytest.approx(0.6 / 1.4)
    assert oracle.chroma_project(0.3, 0.4) == (0.3, 0.4)


@pytest.mark.parametrize("T", [1500.0, 2500.0, 4000.0, 6500.0, 12000.0, 30000.0])
def test_blackbody_colours_shift_like_the_blackbody_at_DT(T):
    """Blackbody colour (band chromaticity of B_T): temperature T back, no absorption, and
    C_b(D) = L_b(D T) / sum L(T) for red and blue shifts."""
    r, g, _ = bb_chroma(T)
    Tc, a1, a2 = oracle.spectrum_of(r, g)
    assert Tc == pytest.approx(T, rel=1e-9)
    assert abs(a1) < 1e-7 and abs(a2) < 1e-7
    S = bands_of(lambda l: planck(l, T)).sum()
    for D in (0.2, 0.7, 1.3, 3.5):
        want = bands_of(lambda l: planck(l, D * T)) / S
        got = oracle.color_shift(r, g, D)
        assert np.allclose(got, want, rtol=1e-8, atol=0.0), (D, got, want)


@pytest.mark.parametrize("rg", in_gamut_grid())
def test_the_chosen_spectrum_has_the_requested_colour(rg):
    """The spectrum B_T (1 - a1 A1 - a2 A2) has band chromaticity (r, g), integrated here;
    its temperature has the blue-to-red ratio b / r; and C(r, g, 1) = (r, g, b)."""
    r, g = rg
    b = 1.0 - r - g
    T, a1, a2 = oracle.spectrum_of(r, g)
    I = bands_of(lambda l: planck(l, T) * (1.0 - a1 * gauss(l, 450e-9) - a2 * gauss(l, 650e-9)))
    assert np.allclose(I / I.sum(), [r, g, b], rtol=0.0, atol=1e-10)
    L = bands_of(lambda l: planck(l, T))
    assert L[2] / L[0] == pytest.approx(b / r, rel=1e-9)
    assert np.allclose(oracle.color_shift(r, g, 1.0), [r, g, b], rtol=0.0, atol=1e-12)


def test_correlated_temperature_clamps_and_order():
    assert oracle.band_cct(0.95, 0.05) == 1000.0           # b = 0: reddest
    assert oracle.band_cct(0.0, 0.3) == 1.0e6              # r = 0: bluest
    Ts = [oracle.band_cct(r, 0.3) for r in (0.6, 0.5, 0.4, 0.3, 0.2, 0.15)]
    assert all(a < b for a, b in zip(Ts, Ts[1:]))          # bluer -> hotter


def test_out_of_gamut_colours_keep_a_non_negative_spectrum():
    """A colour far from the blackbody locus needs more than full absorption: the
    coefficients stop at 1 and the spectrum stays non-negative."""
    T, a1, a2 = oracle.spectrum_of(0.2, 0.7)
    assert a1 == 1.0 or a2 == 1.0
    lam = np.linspace(200e-9, 6000e-9, 5801)
    s = np.array([1.0 - a1 * oracle.absorption(0, l) - a2 * oracle.absorption(1, l) for l in lam])
    assert s.min() >= -1e-9
    assert (oracle.color_shift(0.2, 0.7, 1.0) >= 0.0).all()


def test_table_nodes_and_interpolation():
    n = 9
    tab = oracle.cshift_table(n, n, n)
    for (i, j, k) in ((0, 0, 0), (2, 3, 4), (4, 2, 8), (8, 0, 5), (3, 3, 0)):
        r, g, D = i / (n - 1), j / (n - 1), 2.0 ** (-3 + 6 * k / (n - 1))
        want = np.log2(np.maximum(oracle.color_shift(r, g, D), 2.0 ** -100))
        assert np.allclose(tab[i, j, k], want, rtol=0.0, atol=1e-12)
        assert np.allclose(oracle.cshift_lookup(tab, r, g, D), 2.0 ** tab[i, j, k], rtol=1e-14)
    # linear in r (log2 values) between nodes, D and g on nodes
    i, j, k = 3, 4, 5
    D = 2.0 ** (-3 + 6 * k / (n - 1))
    got = oracle.cshift_lookup(tab, (i + 0.25) / (n - 1), j / (n - 1), D)
    assert np.allclose(np.log2(got), 0.75 * tab[i, j, k] + 0.25 * tab[i + 1, j, k], atol=1e-12)
    # linear in 1 / D between the D nodes
    d0, d1 = 2.0 ** (-3 + 6 * k / (n - 1)), 2.0 ** (-3 + 6 * (k + 1) / (n - 1))
    D = 1.0 / (0.6 / d0 + 0.4 / d1)
    got = oracle.cshift_lookup(tab, i / (n - 1), j / (n - 1), D)
    assert np.allclose(np.log2(got), 0.6 * tab[i, j, k] + 0.4 * tab[i, j, k + 1], atol=1e-12)
    # clamped coordinates
    assert np.array_equal(oracle.cshift_lookup(tab, 0.3, 0.3, 100.0),
                          oracle.cshift_lookup(tab, 0.3, 0.3, 8.0))
    assert np.array_equal(oracle.cshift_lookup(tab, -1.0, 0.3, 1.0),
                          oracle.cshift_lookup(tab, 0.0, 0.3, 1.0))


@pytest.fixture(scope="module")
def full_table():
    return oracle.cshift_table(*oracle.CSHIFT_DIMS)


def test_table_against_the_exact_shift(full_table):
    """The 128^3 table against the exact shift on the colours the seeded band maps use
    (r in [0.15, 0.55], g in [0.2, 0.45]) and D from 0.2 to 5, relative to the largest
    band: measured p50 4.5e-4, p90 3.6e-3, p99 9e-3."""
    rng = np.random.default_rng(5)
    errs = []
    while len(errs) < 400:
        r, g = rng.uniform(0.15, 0.55), rng.uniform(0.2, 0.45)
        if r + g > 0.95:
            continue
        D = 2.0 ** rng.uniform(math.log2(0.2), math.log2(5.0))
        ex = oracle.color_shift(r, g, D)
        lk = oracle.cshift_lookup(full_table, r, g, D)
        errs.append(np.abs(lk - ex).max() / ex.max())
    p50, p90, mx = np.percentile(errs, [50, 90, 100])
    assert p50 < 1.5e-3 and p90 < 8e-3 and mx < 5e-2, (p50, p90, mx)
