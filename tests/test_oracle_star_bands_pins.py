"""Pins of the oracle's band-colour star map (stars of any colour, received through the
colour shift of Section 3.4.2; oracle/emission.c, oracle/render.c): band sums conserved
by the mip rule, a lone star's direction recovered from its stored position at every
level, the merge rule of two stars in one texel, and the render: a field of stars of one
temperature gives the same light as band colours (exact shift) as through the (I, T) map,
since the band model shifts a blackbody's colour to the blackbody at D T."""
import math

import numpy as np
import pytest
import scipy.integrate as si

from paper_2010_08735_amd import scenes

EDGES = [700e-9, 600e-9, 500e-9, 400e-9]


def _texel_direction(face, tx, ty, pu, pv, n):
    k, sgn = face // 2, (-1.0 if face % 2 else 1.0)
    U = 2.0 * (tx + pu) / n - 1.0
    V = 2.0 * (ty + pv) / n - 1.0
    d = np.zeros(3)
    d[k] = sgn
    d[(k + 1) % 3] = U
    d[(k + 2) % 3] = V
    return d / np.linalg.norm(d)


def _face_uv(d):
    k = int(np.argmax(np.abs(d)))
    return 2 * k + (d[k] < 0), d[(k + 1) % 3] / abs(d[k]), d[(k + 2) % 3] / abs(d[k])


def test_band_sums_are_conserved_per_level(orc):
    rng = np.random.default_rng(3)
    f = scenes.star_field(3000, 8)
    rgb = (f.intensity[:, None] * rng.uniform(0.1, 1.0, (3000, 3))).astype(np.float32)
    n0 = 64
    tex = orc.cubemap_bands(f.dirs, rgb, n0)
    tot = rgb.astype(np.float64).sum(axis=0)
    for L in range(7):
        lv = orc.cubemap_level_bands(tex, n0, L)
        assert np.allclose(lv[..., :3].reshape(-1, 3).sum(axis=0), tot, rtol=1e-12)


def test_lone_star_position_at_every_level(orc):
    n0 = 64
    rng = np.random.default_rng(12)
    for _ in range(10):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = np.array([[0.2, 0.5, 0.3]], np.float32)
        tex = orc.cubemap_bands(d[None, :].astype(np.float32), c, n0)
        d64 = d.astype(np.float32).astype(np.float64)
        d64 /= np.linalg.norm(d64)
        face, U, V = _face_uv(d64)
        for L in range(7):
            nl = n0 >> L
            lv = orc.cubemap_level_bands(tex, n0, L)
            tx, ty = int((U + 1) / 2 * nl), int((V + 1) / 2 * nl)
            t = lv[face, ty, tx]
            assert np.allclose(t[:3], c[0].astype(np.float64), rtol=1e-12)
            assert np.allclose(_texel_direction(face, tx, ty, t[3], t[4], nl), d64, atol=1e-12)


def test_two_stars_in_one_texel_merge_by_band_sums(orc):
    """Two stars in one level-0 texel: the texel holds their band sums and their position
    weighted by each star's band sum S (numpy, from the face coordinates)."""
    n0 = 16
    a = np.array([0.101, -0.052, 1.0])
    b = np.array([0.104, -0.049, 1.0])
    dirs = np.stack([a / np.linalg.norm(a), b / np.linalg.norm(b)]).astype(np.float32)
    c = np.array([[0.3, 0.1, 0.05], [0.02, 0.2, 0.4]], np.float32)
    tex = orc.cubemap_bands(dirs, c, n0)
    lv = orc.cubemap_level_bands(tex, n0, 0)
    pos = []
    for d in dirs.astype(np.float64):
        d = d / np.linalg.norm(d)
        face, U, V = _face_uv(d)
        gx, gy = 0.5 * (U + 1) * n0, 0.5 * (V + 1) * n0
        pos.append((face, int(gx), int(gy), gx - int(gx), gy - int(gy)))
    assert pos[0][:3] == pos[1][:3]
    face, tx, ty = pos[0][:3]
    S = c.astype(np.float64).sum(axis=1)
    t = lv[face, ty, tx]
    assert np.allclose(t[:3], c.astype(np.float64).sum(axis=0), rtol=1e-12)
    assert t[3] == pytest.approx((S[0] * pos[0][3] + S[1] * pos[1][3]) / S.sum(), abs=1e-12)
    assert t[4] == pytest.approx((S[0] * pos[0][4] + S[1] * pos[1][4]) / S.sum(), abs=1e-12)


def test_rejects_negative_and_infinite_bands(orc):
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    for bad in ([-0.1, 0.2, 0.3], [0.1, np.inf, 0.3]):
        with pytest.raises(ValueError):
            orc.cubemap_bands(d, np.array([bad], np.float32), 8)


def test_one_temperature_field_renders_alike_as_bands_and_as_temperatures(orc):
    """Stars of one temperature T: the band map (R, G, B) = I L_b(T) / sum L(T) received with
    the exact colour shift gives each pixel the light of the (I, T) map, star pixel by star
    pixel (merged texels keep the same T and the same chromaticity)."""
    T = 6500.0
    L = np.array([si.quad(lambda l: orc.planck(l, T), EDGES[b + 1], EDGES[b],
                          epsabs=0, epsrel=1e-13)[0] for b in range(3)])
    chroma = L / L.sum()
    f = scenes.star_field(4000, 9)
    f = scenes.StarField(f.dirs, f.intensity, np.full(len(f), T, np.float32), 0)
    rgb = (f.intensity.astype(np.float64)[:, None] * chroma[None, :]).astype(np.float32)
    n0 = 64
    cube_t = orc.cubemap(f, n0)
    cube_b = orc.cubemap_bands(f.dirs, rgb, n0)
    v = scenes.small_static_view()
    v.width = v.height = 48
    v.disc_opacity = 0.0
    v.cam_vel = tuple(0.4 * scenes.azimuthal_direction(np.array(v.cam_pos)))
    q = scenes.all_quads(48, 48)
    pt = orc.render_quads(v, q, cube=cube_t, n0=n0)
    pb = orc.render_quads(v, q, cube=cube_b, n0=n0, star_bands=True)
    lit = pt["star_A"] > 0
    assert lit.sum() > 300
    assert np.allclose(pb["star_A"], pt["star_A"], rtol=1e-6)
    # band sums are float32 copies of I times the chromaticity: 1e-6 relative
    r = np.abs(pb["star_rgb"][lit] - pt["star_rgb"][lit]).max(axis=1) / pt["star_rgb"][lit].max(axis=1)
    assert r.max() < 2e-6, r.max()
    assert np.all(pb["star_rgb"][~lit] == 0.0)
