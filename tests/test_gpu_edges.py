"""Degenerate and extreme configurations of the method against the oracle: an empty star
field, a camera on the disc's axis (every beam plane's line of nodes at alpha = pi/2), an
edge-on camera whose middle row of beams lies in the disc plane, a far camera (r = 1000)
and a camera just outside the horizon (r = 1.1).  Same tolerances and mask as the 128x128
full-frame test; the mask is wider where degenerate beam planes are the point."""
import json
import math

import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

import parity

pytestmark = pytest.mark.gpu


def _report(s):
    print("\nPARITY " + json.dumps(s, sort_keys=True))


def _full_frame(gpu_ctx, gpu_tables, orc, orc_tables, v, scene, name, masked=0.02,
                masked_exact=0.02):
    field, n0, h, cube = scene
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    assert np.isfinite(rgb).all() and np.all(rgb[..., 3] == 1.0)
    quads = scenes.all_quads(v.width, v.height)
    quads = quads[(quads[:, 0] + 1 < v.width) & (quads[:, 1] + 1 < v.height)]
    pt = orc.render_quads(v, quads, cube=cube, n0=n0, tables=orc_tables)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    g = parity.gpu_at(rgb, aov, pt)
    st, se = parity.compare(pt, g, "table"), parity.compare(pe, g, "exact")
    _report({name + "_table": st, name + "_exact": se})
    assert st["finite"] and st["masked_fraction"] < masked
    assert se["masked_fraction"] < masked_exact
    assert st["dprime_max"] < 5e-4 and st["u_max"] < 2e-4
    assert se["dprime_max"] < 1e-3 and se["u_max"] < 1e-3
    assert parity.frac_within(pt, g, 1e-3, "disc") > 0.995
    assert parity.frac_within(pt, g, 2e-2, "star") > 0.99
    assert parity.frac_within(pt, g, 2e-2, "all") > 0.995
    return pt, g


def test_empty_star_field_adds_nothing(gpu_ctx, gpu_tables):
    """A star map built from no stars: every texel empty, so each pixel equals the render
    without a star map, bit for bit."""
    field = scenes.StarField(np.zeros((0, 3), np.float32), np.zeros(0, np.float32),
                             np.zeros(0, np.float32), 0)
    from conftest import gpu_star_map
    h = gpu_star_map(gpu_ctx, field, 64, bh.BH_TEXEL_FP16)
    v = scenes.small_static_view()
    with_map, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    without, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, None)
    assert np.array_equal(with_map, without)
    assert (without[..., :3] > 0).any()  # the disc is there


def test_camera_on_the_disc_axis(gpu_ctx, gpu_tables, orc, orc_tables, small_scene):
    """Camera on +z at r = 15 looking at the hole: the disc face-on, every beam plane
    contains the axis, so its line of nodes is perpendicular to it (alpha = pi/2).  The
    disc's inner and outer edges are whole circles across the image, and against exact
    geodesics the crossing count flips wherever the method's crossing error (u within
    2.5e-4) straddles u_ic or u_oc: those pixels are masked, up to 5% here (none against
    the method in FP64)."""
    v = scenes.aimed_view(np.array([0.0, 0.0, 15.0]), np.zeros(3), 64, 64,
                          fov_y=math.radians(90.0), disc_r_in=3.0, disc_r_out=12.0)
    pt, g = _full_frame(gpu_ctx, gpu_tables, orc, orc_tables, v, small_scene, "axis",
                        masked_exact=0.05)
    assert np.allclose(pt["alpha"][pt["captured"] == 0], math.pi / 2, atol=1e-9)
    assert (pt["n_cross"] > 0).mean() > 0.3  # the face-on disc fills much of the view


def test_edge_on_camera(gpu_ctx, gpu_tables, orc, orc_tables, small_scene):
    """Camera in the disc plane; with an odd height the middle row's beams lie in that plane
    (degenerate line of nodes: flagged, no crossing) and the disc is a thin line."""
    v = scenes.aimed_view(scenes.spherical_position(15.0, math.pi / 2, 0.3), np.zeros(3),
                          64, 63, fov_y=math.radians(60.0), disc_r_in=3.0, disc_r_out=12.0)
    pt, g = _full_frame(gpu_ctx, gpu_tables, orc, orc_tables, v, small_scene, "edge_on",
                        masked=0.06, masked_exact=0.06)
    assert (pt["n_cross"] > 0).any()


def test_far_camera(gpu_ctx, gpu_tables, orc, orc_tables, small_scene):
    """Camera at r = 1000 with a 0.02 rad field: u = 1e-3, the shadow (radius 2.6e-3 rad)
    about 17 pixels wide, the disc [3, 20] seen 80 degrees from its axis."""
    v = scenes.aimed_view(scenes.spherical_position(1000.0, math.radians(80.0), 1.0),
                          np.zeros(3), 64, 64, fov_y=0.02, disc_r_in=3.0, disc_r_out=20.0)
    pt, g = _full_frame(gpu_ctx, gpu_tables, orc, orc_tables, v, small_scene, "far")
    cap = (pt["captured"] != 0).mean()
    assert 0.01 < cap < 0.3, cap


def test_camera_just_outside_the_horizon(gpu_ctx, gpu_tables, orc, orc_tables, small_scene):
    """Static camera at r = 1.1 (u = 0.91) looking straight out: light escapes only inside a
    cone of half-angle ~45 degrees (Synge), the rest of the 120-degree view is shadow."""
    pos = scenes.spherical_position(1.1, math.radians(60.0), 0.7)
    out = pos / np.linalg.norm(pos)
    v = scenes.View(cam_pos=tuple(float(x) for x in pos), cam_vel=(0.0, 0.0, 0.0),
                    cam_rot=scenes.look_rotation(out), width=64, height=64,
                    fov_y=math.radians(120.0), disc_r_in=3.0, disc_r_out=12.0)
    pt, g = _full_frame(gpu_ctx, gpu_tables, orc, orc_tables, v, small_scene, "horizon")
    cap = (pt["captured"] != 0).mean()
    assert 0.2 < cap < 0.9, cap


def test_generic_release_frees_every_handle_type(gpu_ctx):
    """bh_release frees tables, star maps, area maps, particles and bloom pyramids like the
    typed release calls: the context's device bytes return to where they were, and a
    second release of the same address is refused."""
    import torch
    from conftest import gpu_star_map
    ctx = bh.bh_create(0, 0)
    try:
        base = bh.bh_bytes_in_use(ctx)
        field = scenes.star_field(2000, 5)
        it = scenes.area_map(16, 3)
        t = torch.from_numpy(np.ascontiguousarray(it, np.float32)).cuda()
        handles = [
            bh.bh_precompute_tables(ctx, d_n=64, u_ne=16, u_nphi=8),
            gpu_star_map(ctx, field, 32, bh.BH_TEXEL_FP16),
            bh.bh_build_area(ctx, t.data_ptr(), 16, bh.current_stream()),
            bh.bh_create_particles(ctx, [[6.0, 9.0, 0.5], [4.0, 4.0, 1.0]]),
            bh.bh_bloom_create(ctx, 64, 32, 3),
        ]
        torch.cuda.synchronize()
        assert bh.bh_bytes_in_use(ctx) > base
        for h in handles:
            bh.bh_release(h)
        assert bh.bh_bytes_in_use(ctx) == base
        for h in handles:
            with pytest.raises(bh.BhError) as e:
                bh.bh_release(h)
            assert e.value.status == bh.BH_EINVAL
    finally:
        bh.bh_destroy(ctx)


def test_opaque_disc_hides_stars_and_area_exactly(gpu_ctx, gpu_tables, small_scene):
    """Behind an opaque disc crossing (transmittance exactly 0) star and area light are
    multiplied by 0, which lets the kernel skip their gather and filter: every pixel with a
    crossing has the same bits with and without the star map and area sky, pixels without
    one do not; a semi-transparent disc lets star light through, so there the two differ."""
    import torch
    field, n0, h, cube = small_scene
    it = scenes.area_map(32, 21)
    t = torch.from_numpy(np.ascontiguousarray(it)).cuda()
    ah = bh.bh_build_area(gpu_ctx, t.data_ptr(), 32, bh.current_stream())
    torch.cuda.synchronize()
    try:
        v = scenes.boosted_orbit_view(256, 144)
        v.k_area = 0.5
        with_sky, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h, area=ah)
        bare, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, None)
        bits = aov[..., 3].copy().view(np.uint32)
        cross = (bits & 6) != 0
        assert cross.mean() > 0.3 and (~cross).mean() > 0.2
        assert np.array_equal(with_sky[cross].view(np.uint32), bare[cross].view(np.uint32))
        assert (with_sky[~cross, :3] != bare[~cross, :3]).any(axis=1).mean() > 0.9
        v.disc_opacity = 0.5
        half_sky, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, h, area=ah)
        half_bare, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, None)
        seen = (half_sky[cross, :3] != half_bare[cross, :3]).any(axis=1)
        assert seen.mean() > 0.9
    finally:
        bh.bh_release_area(ah)
