"""Pins of the oracle's area-source functions (Section 3.3.2 "Emitted light": nebulae and
galaxies in a cube map read over the beam's footprint; Section 3.4.1: no lensing
amplification for them).

Expected values come from closed forms, numpy block means, brute-force sampling written
here, and scipy quadrature of Planck's law; none reuse the oracle's code."""
import math

import numpy as np
import pytest
import scipy.integrate as si

from paper_2010_08735_amd import scenes


def _face_of(p):
    """face and (U, V) of a direction: k = argmax |p_k| (lowest index on ties)."""
    k = int(np.argmax(np.abs(p)))
    m = abs(p[k])
    return 2 * k + (1 if p[k] < 0 else 0), p[(k + 1) % 3] / m, p[(k + 2) % 3] / m


def _nearest(level0, p):
    n0 = level0.shape[1]
    f, U, V = _face_of(p)
    i = min(max(int(math.floor((U + 1) / 2 * n0)), 0), n0 - 1)
    j = min(max(int(math.floor((V + 1) / 2 * n0)), 0), n0 - 1)
    return level0[f, j, i]


def _levels_from(it):
    """(6, n0, n0, 2) (I, T) -> list of (6, nL, nL, 2) (I, I T) block means, by numpy."""
    it = it.astype(np.float64)
    lv = [np.stack([it[..., 0], it[..., 0] * it[..., 1]], axis=-1)]
    while lv[-1].shape[1] > 1:
        a = lv[-1]
        n = a.shape[1] // 2
        lv.append(a.reshape(6, n, 2, n, 2, 2).mean(axis=(2, 4)))
    return lv


def _random_map(n0, seed):
    rng = np.random.default_rng(seed)
    it = np.empty((6, n0, n0, 2), np.float32)
    it[..., 0] = rng.uniform(0.1, 2.0, (6, n0, n0))
    it[..., 1] = rng.uniform(3000.0, 12000.0, (6, n0, n0))
    return it


def _footprint(rng, n0, size_lo, size_hi, ani_hi):
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    e1 = np.cross(d, rng.normal(size=3))
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    size = 10 ** rng.uniform(math.log10(size_lo), math.log10(size_hi)) * 2.0 / n0
    ani = 10 ** rng.uniform(0.0, math.log10(ani_hi))
    th = rng.uniform(0.0, math.pi)
    dw = size * ani * (math.cos(th) * e1 + math.sin(th) * e2)
    dh = size * (-math.sin(th) * e1 + math.cos(th) * e2 + rng.uniform(-0.5, 0.5) * e1)
    return d, dw, dh


def test_area_mips_are_block_means(orc):
    it = _random_map(8, 1)
    lv = orc.area_levels(it)
    ref = _levels_from(it)
    for L in range(4):
        assert np.allclose(orc.area_level(lv, 8, L), ref[L], rtol=1e-12, atol=0)


def test_area_exact_of_a_constant_map_is_that_constant(orc):
    """The texel pieces partition the footprint: their areas add up to 1 for footprints of
    every size, including ones over cube edges and corners and ones wrapping most of the
    sphere."""
    n0 = 8
    it = np.empty((6, n0, n0, 2), np.float32)
    it[..., 0] = 0.75
    it[..., 1] = 5000.0
    lv = orc.area_levels(it)
    rng = np.random.default_rng(2)
    for _ in range(60):
        d, dw, dh = _footprint(rng, n0, 0.05, 40.0, 6.0)
        A, B = orc.area_exact(lv, n0, d, dw, dh)
        assert abs(A - 0.75) < 1e-12 and abs(B - 0.75 * 5000.0) < 1e-8
    # a cube corner, where three faces meet
    d = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    A, B = orc.area_exact(lv, n0, d, np.array([0.3, -0.2, 0.0]), np.array([0.0, 0.25, -0.3]))
    assert abs(A - 0.75) < 1e-12


def test_area_exact_inside_one_texel(orc):
    n0 = 16
    it = _random_map(n0, 3)
    lv = orc.area_levels(it)
    # centre of texel (x, y) = (5, 9) on face 4 (+z): U = (5.5) 2/16 - 1, V = (9.5) 2/16 - 1
    U, V = 5.5 * 2 / n0 - 1, 9.5 * 2 / n0 - 1
    d = np.array([U, V, 1.0])      # face 4: k = 2, a = x, b = y
    eps = 0.01 * 2 / n0
    A, B = orc.area_exact(lv, n0, d, np.array([eps, 0.0, 0.0]), np.array([0.0, eps, 0.0]))
    I, T = it[4, 9, 5]
    assert abs(A - I) < 1e-6 * I and abs(B - I * T) < 1e-6 * I * T


@pytest.mark.parametrize("w0", [0.0, 0.13, -0.31])
def test_area_exact_split_across_a_cube_edge(orc, w0):
    """Faces +x (0) and +z (4) uniform at a and b.  Around the edge direction (1, 0, 1) a
    footprint d + w dw + h dh with dw = s (-1, 0, 1) and a small dh along y has
    p_x = c_x - w s, p_z = c_z + w s, so the faces meet at w0 = (c_x - c_z) / (2 s): the
    +z share of the unit square is 1/2 - w0."""
    n0 = 8
    it = np.empty((6, n0, n0, 2), np.float32)
    it[..., 0] = 1.0
    it[..., 1] = 4000.0
    a, b = 0.375, 1.625          # exact in float32
    it[0, ..., 0] = a
    it[4, ..., 0] = b
    lv = orc.area_levels(it)
    s = 0.05
    cz = 0.7
    cx = cz + 2 * s * w0
    d = np.array([cx, 0.0, cz])
    A, _ = orc.area_exact(lv, n0, d, np.array([-s, 0.0, s]), np.array([0.0, 0.02, 0.0]))
    frac_z = 0.5 - w0
    assert abs(A - (frac_z * b + (1 - frac_z) * a)) < 1e-12


def test_area_exact_matches_brute_force_sampling(orc):
    """Against midpoint sampling of the nearest-texel map on a 600 x 600 grid over
    (w, h): a sample differs from the exact mean's texel only where a texel edge crosses
    its cell, so the difference is bounded by (cells on edges) / 600^2 x (largest jump)."""
    n0 = 8
    it = _random_map(n0, 4)
    lv = orc.area_levels(it)
    lv0 = _levels_from(it)[0]
    rng = np.random.default_rng(5)
    ns = 600
    g = (np.arange(ns) + 0.5) / ns - 0.5
    for _ in range(6):
        d, dw, dh = _footprint(rng, n0, 0.5, 6.0, 3.0)
        A, B = orc.area_exact(lv, n0, d, dw, dh)
        P = d[None, None, :] + g[:, None, None] * dw + g[None, :, None] * dh
        vals = np.array([_nearest(lv0, p) for p in P.reshape(-1, 3)])
        ref = vals.mean(axis=0)
        assert abs(A - ref[0]) < 2e-2 * ref[0] and abs(B - ref[1]) < 2e-2 * ref[1]
        # a finer check on the sampling error scale: ~1.9 / 600 per texel edge crossed
        assert abs(A - ref[0]) < 0.05 * 1.9 * 6 / ns * 40


def test_area_filter_of_a_constant_map(orc):
    n0 = 16
    it = np.empty((6, n0, n0, 2), np.float32)
    it[..., 0] = 1.25
    it[..., 1] = 7000.0
    lv = orc.area_levels(it)
    rng = np.random.default_rng(6)
    for _ in range(40):
        d, dw, dh = _footprint(rng, n0, 0.05, 60.0, 10.0)
        A, B = orc.area_filter(lv, n0, d, dw, dh)
        assert abs(A - 1.25) < 1e-12 and abs(B - 1.25 * 7000.0) < 1e-8


def test_area_filter_reproduces_maps_linear_in_face_coordinates(orc):
    """On face +z let I = a + b U + c V at texel centres.  Every mip level then holds the
    same linear function at its own texel centres, bilinear reads reproduce it, and probes
    symmetric about d with footprint axes parallel to the face (zero z component) keep U and
    V affine in the probe offset: the filtered mean is a + b U(d) + c V(d) exactly."""
    n0 = 32
    a, b, c, T0 = 1.0, 0.3, -0.2, 6500.0
    it = np.full((6, n0, n0, 2), 1.0, np.float32)
    cc = (np.arange(n0) + 0.5) * 2 / n0 - 1
    uu, vv = np.meshgrid(cc, cc, indexing="xy")
    it[4, ..., 0] = a + b * uu + c * vv
    it[..., 1] = T0
    lv = orc.area_levels(it.astype(np.float64).astype(np.float32))
    lin = orc.area_level(lv, n0, 0)[4, ..., 0]
    assert np.allclose(lin, a + b * uu + c * vv, rtol=1e-6)   # float32 input
    rng = np.random.default_rng(7)
    for _ in range(30):
        U, V = rng.uniform(-0.3, 0.3, 2)
        d = np.array([U, V, 1.0])
        th = rng.uniform(0, math.pi)
        L1, L2 = rng.uniform(0.3, 3.0, 2) * 2 / n0
        dw = L1 * np.array([math.cos(th), math.sin(th), 0.0])
        dh = L2 * np.array([-math.sin(th), math.cos(th), 0.0]) + 0.3 * dw
        A, B = orc.area_filter(lv, n0, d, dw, dh)
        # the float32 texel values carry ~6e-8 relative rounding
        assert abs(A - (a + b * U + c * V)) < 1e-6
        assert abs(B - T0 * A) < 1e-6 * T0


def test_area_filter_level_of_detail(orc):
    """A checkerboard level 0 has every level >= 1 uniform at 1/2.  An isotropic footprint
    8 level-0 texels wide takes N_maj = 2 probes and lambda = log2(8 / 2) - 1 = 1: level 1
    only, hence exactly 1/2.  A footprint 0.2 texels wide takes a single probe (probes are
    spaced no closer than half a level-0 texel): at a texel's centre it reads exactly that
    texel's 0 or 1 from level 0."""
    n0 = 32
    it = np.empty((6, n0, n0, 2), np.float32)
    ii, jj = np.meshgrid(np.arange(n0), np.arange(n0), indexing="xy")
    it[..., 0] = ((ii + jj) % 2)[None].astype(np.float32)
    it[..., 1] = 5000.0
    lv = orc.area_levels(it)
    d = np.array([17.5 * 2 / n0 - 1, 12.5 * 2 / n0 - 1, 1.0])   # centre of texel (17, 12)
    for width in (8.0, 16.0):
        s = width * 2 / n0
        A, _ = orc.area_filter(lv, n0, d, np.array([s, 0, 0]), np.array([0, s, 0]))
        assert abs(A - 0.5) < 1e-12, (width, A)
    s = 0.2 * 2 / n0
    A, _ = orc.area_filter(lv, n0, d, np.array([s, 0, 0]), np.array([0, s, 0]))
    assert A == 1.0, A      # texel (17, 12): (17 + 12) % 2 = 1


def test_area_filter_is_close_to_the_exact_mean_on_smooth_maps(orc):
    """The filter approximates the exact mean.  On the seeded nebula sky (Gaussian patches
    of 6-20 degrees on 2.8-degree texels) and footprints of 0.2-8 texels with up to 4:1
    anisotropy, the relative difference stays below 2% for 90% of footprints and below 12%
    for all of them.  The largest differences are at sub-texel footprints, where the exact
    mean is one texel's value and the filter's bilinear read interpolates towards the
    neighbours (half a texel of the map's gradient)."""
    n0 = 32
    it = scenes.area_map(n0, 11)
    lv = orc.area_levels(it)
    rng = np.random.default_rng(8)
    err = []
    for _ in range(150):
        d, dw, dh = _footprint(rng, n0, 0.2, 8.0, 4.0)
        A, _ = orc.area_filter(lv, n0, d, dw, dh)
        E, _ = orc.area_exact(lv, n0, d, dw, dh)
        err.append(abs(A - E) / E)
    err = np.array(err)
    assert np.percentile(err, 90) < 2e-2 and err.max() < 1.2e-1, (np.percentile(err, 90), err.max())


def _band_ref(orc, T):
    edges = [700e-9, 600e-9, 500e-9, 400e-9]
    return np.array([si.quad(lambda l: orc.planck(l, T), edges[b + 1], edges[b],
                             epsabs=0, epsrel=1e-12)[0] for b in range(3)])


def test_area_light_in_the_render(orc):
    """A uniform sky of radiance I at temperature T: every pixel of a quad with no captured
    member reads I and T back, and receives k_area I L_b(D_cam T) / sum_b L_b(T) with no
    lensing factor (Section 3.4.1); quads with a captured member get nothing."""
    n0 = 16
    it = np.empty((6, n0, n0, 2), np.float32)
    I, T = 0.5, 6000.0
    it[..., 0] = I
    it[..., 1] = T
    lv = orc.area_levels(it)
    v = scenes.aimed_view(np.array([0.0, -15.0, 2.0]), np.zeros(3), 48, 48,
                          fov_y=math.radians(60), disc_opacity=0.0)
    v.k_area = 2.0
    px = orc.render_quads(v, scenes.all_quads(48, 48), area=lv, area_n0=n0)
    lit = px["star_zeroed"] == 0
    assert lit.sum() > 500 and (~lit).sum() > 50
    assert np.allclose(px["area_A"][lit], I, rtol=1e-12)
    assert np.allclose(px["area_T"][lit], T, rtol=1e-12)
    assert np.all(px["area_rgb"][~lit] == 0)
    norm = _band_ref(orc, T).sum()
    for p in px[lit][::37]:
        ref = v.k_area * I * _band_ref(orc, p["d_cam"] * T) / norm
        assert np.allclose(p["area_rgb"], ref, rtol=1e-9, atol=0)
        assert np.allclose(p["rgb"], p["area_rgb"], rtol=1e-12)   # transparent disc, no stars


# ---- band maps: (R, G, B) per texel, shifted with the colour-shift table (Section 3.4.2) ----

def _random_band_map(n0, seed):
    rng = np.random.default_rng(seed)
    m = np.zeros((6, n0, n0, 4), np.float32)
    m[..., :3] = rng.uniform(0.05, 1.5, (6, n0, n0, 3))
    m[..., 3] = rng.uniform(-5.0, 5.0, (6, n0, n0))   # ignored
    return m


def test_band_map_mips_are_block_means(orc):
    m = _random_band_map(8, 11)
    lv = orc.area_levels_bands(m)
    a = m[..., :3].astype(np.float64)
    for L in range(4):
        assert np.allclose(orc.area_level_bands(lv, 8, L), a, rtol=1e-12, atol=0)
        n = a.shape[1] // 2
        if n:
            a = a.reshape(6, n, 2, n, 2, 3).mean(axis=(2, 4))


def test_band_filter_and_exact_mean_act_on_each_band(orc):
    """The band filter and exact mean are the same linear operators as on the (I, I T)
    maps, applied to each band: a band map whose channels are copies of the radiance and
    of I T channels gives the same numbers."""
    n0 = 8
    it = _random_map(n0, 12)
    lv2 = orc.area_levels(it)
    m = np.zeros((6, n0, n0, 4), np.float32)
    m[..., 0] = it[..., 0]
    m[..., 1] = it[..., 0] * it[..., 1] * 1e-4
    m[..., 2] = it[..., 0]
    lv3 = orc.area_levels_bands(m)
    rng = np.random.default_rng(13)
    for _ in range(20):
        d, dw, dh = _footprint(rng, n0, 0.2, 8.0, 4.0)
        A, B = orc.area_filter(lv2, n0, d, dw, dh)
        f = orc.area_filter_bands(lv3, n0, d, dw, dh)
        assert f[0] == pytest.approx(A, rel=1e-12) and f[2] == pytest.approx(A, rel=1e-12)
        assert f[1] == pytest.approx(B * 1e-4, rel=1e-6)    # I T rounded to float32 in m
        A, B = orc.area_exact(lv2, n0, d, dw, dh)
        e = orc.area_exact_bands(lv3, n0, d, dw, dh)
        assert e[0] == pytest.approx(A, rel=1e-12) and e[2] == pytest.approx(A, rel=1e-12)


def test_band_sky_in_the_render(orc):
    """A uniform band sky (R, G, B): every lit pixel reads its band sum and chromaticity
    back and receives k_area S C(r, g, D_cam), exactly (no table) or from the table; a
    blackbody-coloured sky receives what the temperature map gives."""
    n0 = 16
    rgb = np.array([0.3, 0.45, 0.25])
    m = np.zeros((6, n0, n0, 4), np.float32)
    m[..., :3] = rgb
    lv = orc.area_levels_bands(m)
    rgb = m[0, 0, 0, :3].astype(np.float64)
    S = rgb.sum()
    v = scenes.aimed_view(np.array([0.0, -15.0, 2.0]), np.array([0.3, 0.2, 0.0]), 32, 32,
                          fov_y=math.radians(60), disc_opacity=0.0)
    v.k_area = 2.0
    q = scenes.all_quads(32, 32)
    px = orc.render_quads(v, q, area=lv, area_n0=n0, area_bands=True)
    lit = px["star_zeroed"] == 0
    assert lit.sum() > 100 and (~lit).sum() > 10
    assert np.allclose(px["area_A"][lit], S, rtol=1e-12)
    assert np.allclose(px["area_chroma"][lit], rgb[:2] / S, rtol=1e-12)
    assert np.all(px["area_rgb"][~lit] == 0)
    for p in px[lit][::23]:
        ref = v.k_area * S * orc.color_shift(rgb[0] / S, rgb[1] / S, p["d_cam"])
        assert np.allclose(p["area_rgb"], ref, rtol=1e-12, atol=0)
    tab = orc.cshift_table(9, 9, 9)
    pt = orc.render_quads(v, q, area=lv, area_n0=n0, area_bands=True, ctable=tab)
    for p in pt[lit][::23]:
        ref = v.k_area * S * orc.cshift_lookup(tab, rgb[0] / S, rgb[1] / S, p["d_cam"])
        assert np.allclose(p["area_rgb"], ref, rtol=1e-12, atol=0)
    # a blackbody sky as a band map: the exact shift equals the temperature map's light
    T = 5000.0
    L = _band_ref(orc, T)
    mb = np.zeros((6, n0, n0, 4), np.float32)
    mb[..., :3] = (0.5 * L / L.sum()).astype(np.float32)
    it = np.empty((6, n0, n0, 2), np.float32)
    it[..., 0] = mb[0, 0, 0, :3].astype(np.float64).sum()
    it[..., 1] = T
    pb = orc.render_quads(v, q, area=orc.area_levels_bands(mb), area_n0=n0, area_bands=True)
    pT = orc.render_quads(v, q, area=orc.area_levels(it), area_n0=n0)
    assert np.allclose(pb["area_rgb"][lit], pT["area_rgb"][lit], rtol=2e-6, atol=0)
