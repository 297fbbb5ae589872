"""Precision study, edge cases and the systems forms, through the C ABI on the GPU."""
import json
import math
import time

import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

from conftest import gpu_star_map
import parity

pytestmark = pytest.mark.gpu


def _report(s):
    print("\nSTATS " + json.dumps(s, sort_keys=True))


def _download(tables, n):
    D = np.zeros((n, n), np.float32)
    U = np.zeros((32, 64), np.float32)
    bh.bh_tables_download(tables, D.ctypes.data, U.ctypes.data)
    return D, U


def test_precision_study_2048_tables(gpu_ctx, orc):
    """2048x2048 deflection table: FP32 everywhere, FP32 + FP64 photon-sphere band and FP64
    everywhere, each against quadrature at the same texel centres."""
    ref = orc.Tables(2048, 64, 32)
    stats = {}
    for name, prec in (("fp32", bh.BH_TAB_FP32), ("fp64_band", bh.BH_TAB_FP64_BAND),
                       ("fp64_all", bh.BH_TAB_FP64_ALL)):
        t = bh.bh_precompute_tables(gpu_ctx, 2048, 64, 32, prec, 0.05)
        D, U = _download(t, 2048)
        err = np.abs(D - ref.D) / np.maximum(1.0, np.abs(ref.D))
        stats[name] = {"D_max": float(err.max()), "D_mean": float(err.mean()),
                       "D_max_rad": float(np.abs(D - ref.D).max()),
                       "U_max": float(np.abs(U - ref.U).max())}
        bh.bh_release_tables(t)
    _report({"tables_2048": stats})
    assert stats["fp64_band"]["D_max"] < 1e-6 and stats["fp64_all"]["D_max"] < 1e-6
    assert stats["fp64_band"]["U_max"] < 1e-6 and stats["fp64_all"]["U_max"] < 1e-6
    assert stats["fp32"]["D_max"] >= stats["fp64_band"]["D_max"]


def test_precision_study_4k_star_map_formats(gpu_ctx, orc, big_field_scene):
    """3840x2160 render of the boosted-orbit scene through the 2048^2 table with an FP16 and
    an FP32 star map (FP32 accumulation in both), each against the oracle on a seeded 1% of
    the quads."""
    field, n0, h16, cube = big_field_scene
    tables = bh.bh_precompute_tables(gpu_ctx, 2048, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
    ref_tables = orc.Tables(2048, 64, 32)
    v = scenes.boosted_orbit_view(3840, 2160)
    quads = scenes.sample_quads(v.width, v.height, 0.01, 22)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    pt = orc.render_quads(v, quads, cube=cube, n0=n0, tables=ref_tables)
    h32 = gpu_star_map(gpu_ctx, field, n0, bh.BH_TEXEL_FP32)
    out = {}
    try:
        for name, h in (("fp16", h16), ("fp32", h32)):
            rgb, aov = parity.render_gpu(gpu_ctx, tables, v, h)
            assert np.isfinite(rgb).all()
            g = parity.gpu_at(rgb, aov, pe)
            out[name] = {"exact": parity.compare(pe, g, "exact"),
                         "table": parity.compare(pt, g, "table"),
                         "star_within_2e-2": parity.frac_within(pt, g, 2e-2, "star"),
                         "star_within_1e-2": parity.frac_within(pt, g, 1e-2, "star"),
                         "star_within_1e-3": parity.frac_within(pt, g, 1e-3, "star"),
                         "disc_within_1e-3": parity.frac_within(pt, g, 1e-3, "disc")}
            del rgb, aov
    finally:
        bh.bh_release_stars(h32)
        bh.bh_release_tables(tables)
    _report({"render_4k": out})
    for name in ("fp16", "fp32"):
        t, e = out[name]["table"], out[name]["exact"]
        assert t["masked_fraction"] < 0.02 and e["masked_fraction"] < 0.02
        assert t["dprime_max"] < 1e-3 and e["dprime_max"] < 1e-3
        # footprints at 4K are about one level-0 texel wide, so the FP32 deflection error
        # (a few microradians) moves stars inside the tent by ~1% of its radius
        assert out[name]["star_within_2e-2"] > 0.99
        assert out[name]["disc_within_1e-3"] > 0.995
    assert out["fp32"]["star_within_1e-3"] >= out["fp16"]["star_within_1e-3"]
    assert out["fp32"]["star_within_1e-2"] >= out["fp16"]["star_within_1e-2"]


def test_paper_temperature_law_and_black_sky(gpu_ctx, gpu_tables, orc, orc_tables):
    """The T^4 ~ u^3 (1 - sqrt(3u)) law (Section 3.3.3) with no star map: the disc matches
    the oracle and every pixel without a disc crossing is black."""
    v = scenes.small_static_view()
    v.disc_T_law = scenes.T_LAW_PAPER
    v.disc_T0 = 8000.0
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, None)
    pt = orc.render_quads(v, scenes.all_quads(v.width, v.height), tables=orc_tables)
    g = parity.gpu_at(rgb, aov, pt)
    s = parity.compare(pt, g, "table")
    _report({"paper_T_law": s})
    assert s["masked_fraction"] < 0.02
    assert parity.frac_within(pt, g, 1e-3, "disc") > 0.995
    assert np.all(g["rgb"][g["ncross"] == 0] == 0.0)
    assert np.all(g["rgb"][g["ncross"] > 0].max(axis=1) > 0.0)


def test_every_tile_configuration_gives_the_same_image(gpu_ctx, gpu_tables):
    field = scenes.star_field(20000, 0)
    h = gpu_star_map(gpu_ctx, field, 256, bh.BH_TEXEL_FP16)
    v = scenes.boosted_orbit_view(200, 136)   # not a multiple of any tile
    ref = None
    try:
        for k in range(bh.bh_tile_config_count()):
            bh.bh_set_tile_config(gpu_ctx, k)
            img, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, h, aov=False)
            if ref is None:
                ref = img
            assert np.array_equal(img, ref), k
    finally:
        bh.bh_set_tile_config(gpu_ctx, -1)


@pytest.mark.parametrize("W,H", [(1, 1), (3, 5), (17, 9), (130, 66)])
def test_small_and_ragged_images(gpu_ctx, gpu_tables, orc, orc_tables, W, H):
    """Images smaller than a tile and with odd sizes: every pixel is written, capture agrees
    with the oracle and escaping beams carry the same deflection."""
    field = scenes.star_field(20000, 0)
    h = gpu_star_map(gpu_ctx, field, 256, bh.BH_TEXEL_FP16)
    v = scenes.small_static_view()
    v.width, v.height = W, H
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    assert rgb.shape == (H, W, 4) and np.isfinite(rgb).all() and np.isfinite(aov[..., 1:]).all()
    captured = (aov[..., 3].copy().view(np.uint32) & bh.BH_AOV_CAPTURED) != 0
    assert np.all(np.isinf(aov[..., 0][captured])) and np.isfinite(aov[..., 0][~captured]).all()
    pt = orc.render_quads(v, scenes.all_quads(W, H), tables=orc_tables)
    pt = pt[(pt["x"] < W) & (pt["y"] < H)]
    assert len(pt) == W * H
    g = parity.gpu_at(rgb, aov, pt)
    ring = (np.abs(pt["e2_over_mu"] - 1.0) < 1e-3) | (pt["degenerate"] != 0)
    same = ((pt["captured"] != 0) == g["captured"]) & (pt["n_cross"] == g["ncross"])
    if (~ring).any():
        assert same[~ring].mean() > 0.98
    # a beam aimed straight at the hole (the 1x1 image) is radial: captured on both sides
    radial = pt["degenerate"] != 0
    assert np.array_equal(pt["captured"][radial] != 0, g["captured"][radial])
    esc = same & ~ring & (pt["captured"] == 0)
    if esc.any():
        assert np.abs(pt["delta_prime"][esc] - g["dprime"][esc]).max() < 1e-3


def test_camera_between_photon_sphere_and_isco(gpu_ctx, gpu_tables, orc, orc_tables):
    """Camera at r = 2 (inside the disc's inner edge r = 3, outside the photon sphere
    r = 1.5), looking 60 degrees away from the hole: about half the image is the shadow and
    the disc is seen from inside its inner edge."""
    pos = scenes.spherical_position(2.0, math.radians(70), 0.4)
    hole = -pos / np.linalg.norm(pos)
    a = math.radians(60.0)
    look = math.cos(a) * hole + math.sin(a) * scenes.azimuthal_direction(pos)
    v = scenes.View(cam_pos=tuple(float(x) for x in pos), cam_vel=(0.0, 0.0, 0.0),
                    cam_rot=scenes.look_rotation(look), width=96, height=96,
                    fov_y=math.radians(90.0), disc_r_in=3.0, disc_r_out=15.0)
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, None)
    quads = scenes.all_quads(96, 96)
    pt = orc.render_quads(v, quads, tables=orc_tables)
    pe = orc.render_quads(v, quads)
    g = parity.gpu_at(rgb, aov, pt)
    st, se = parity.compare(pt, g, "table"), parity.compare(pe, g, "exact")
    _report({"r2_table": st, "r2_exact": se})
    assert 0.3 < (pt["captured"] != 0).mean() < 0.8 and (pt["n_cross"] > 0).mean() > 0.05
    assert st["masked_fraction"] < 0.03
    assert st["dprime_max"] < 1e-3 and se["dprime_max"] < 1e-3
    assert st["u_max"] < 2e-4
    assert parity.frac_within(pt, g, 1e-3, "disc") > 0.99


def test_tables_and_star_maps_are_shared_by_key(gpu_ctx):
    """Tables are shared by parameters; star maps by content (a hash of the star arrays,
    the star count, the face size and the texel format): the same stars uploaded again
    into new device arrays share the map, a different field of the same size does not,
    and neither does one changed in a single star's temperature."""
    t1 = bh.bh_precompute_tables(gpu_ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
    used = bh.bh_bytes_in_use(gpu_ctx)
    t2 = bh.bh_precompute_tables(gpu_ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
    assert t1 == t2 and bh.bh_bytes_in_use(gpu_ctx) == used
    field = scenes.star_field(5000, 9)
    s1 = gpu_star_map(gpu_ctx, field, 128, bh.BH_TEXEL_FP16)
    used = bh.bh_bytes_in_use(gpu_ctx)
    s2 = gpu_star_map(gpu_ctx, field, 128, bh.BH_TEXEL_FP16)
    assert s1 == s2 and bh.bh_bytes_in_use(gpu_ctx) == used
    s3 = gpu_star_map(gpu_ctx, field, 128, bh.BH_TEXEL_FP32)
    assert s3 != s1 and bh.bh_bytes_in_use(gpu_ctx) > used
    other = scenes.star_field(5000, 10)
    s4 = gpu_star_map(gpu_ctx, other, 128, bh.BH_TEXEL_FP16)
    assert s4 not in (s1, s3)
    tweaked = scenes.StarField(field.dirs, field.intensity, field.temperature.copy(), 0)
    tweaked.temperature[1234] += 1.0
    s5 = gpu_star_map(gpu_ctx, tweaked, 128, bh.BH_TEXEL_FP16)
    assert s5 not in (s1, s3, s4)
    for s in (s5, s4, s3, s2, s1):
        bh.bh_release_stars(s)
    bh.bh_release_tables(t2)
    bh.bh_release_tables(t1)


def _device_to_host(ptr, shape):
    """Copy a library-owned device image into a new host array."""
    import ctypes
    import torch
    host = np.zeros(shape, np.float32)
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(host.ctypes.data, ptr, host.nbytes, 2) == 0  # device to host
    return host


def test_serving_admits_by_hbm_budget(gpu_ctx, gpu_tables):
    """Library-allocated images under a budget that holds two of them: a frame bigger than
    the budget is refused, the rest wait for admission, all complete within the budget, and
    each image equals the plain render."""
    views = [scenes.small_static_view() for _ in range(6)]
    for k, v in enumerate(views):
        v.width, v.height = 256, 160
        v.disc_r_out = 10.0 + k
    img_bytes = 16 * 256 * 160
    probe = bh.bh_create(0, 0)
    try:
        bh.bh_precompute_tables(probe, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        base = bh.bh_bytes_in_use(probe)
    finally:
        bh.bh_destroy(probe)
    budget = base + 2 * img_bytes + 4096
    ctx = bh.bh_create(0, budget)
    images = {}
    try:
        tables = bh.bh_precompute_tables(ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        bh.bh_serve_start(ctx, 0, 2, 16)
        big = scenes.small_static_view()
        big.width, big.height = 4096, 4096
        with pytest.raises(bh.BhError) as ei:
            bh.bh_submit(ctx, tables, bh.make_view(big), None)
        assert ei.value.status == bh.BH_ENOMEM
        tickets = [bh.bh_submit(ctx, tables, bh.make_view(v), None) for v in views]
        deadline = time.time() + 60
        while len(images) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t in images:
                    continue
                done, _ = bh.bh_poll(ctx, t)
                if done:
                    images[t] = _device_to_host(bh.bh_ticket_image(ctx, t), (160, 256, 4))
                    bh.bh_ticket_free(ctx, t)
                    assert bh.bh_bytes_in_use(ctx) <= budget
            time.sleep(0.001)
        assert len(images) == len(tickets)
        with pytest.raises(bh.BhError) as ei:
            bh.bh_poll(ctx, tickets[0])
        assert ei.value.status == bh.BH_ENOTFOUND
    finally:
        bh.bh_destroy(ctx)
    for t, v in zip(tickets, views):
        ref, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, None, aov=False)
        assert np.array_equal(images[t], ref)


def test_serving_fails_a_frame_that_can_never_fit(gpu_tables):
    """A library-allocated image that fits the budget on paper but not beside the resident
    resources, with nothing else holding budget: the request fails with BH_ENOMEM instead of
    waiting forever, and the server keeps serving frames with caller-owned images."""
    import torch
    probe = bh.bh_create(0, 0)
    try:
        bh.bh_precompute_tables(probe, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        base = bh.bh_bytes_in_use(probe)
    finally:
        bh.bh_destroy(probe)
    ctx = bh.bh_create(0, base + 2048)
    try:
        tables = bh.bh_precompute_tables(ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        bh.bh_serve_start(ctx, 0, 2, 64)
        v = scenes.small_static_view()
        v.width, v.height = 16, 16           # 4 KiB image: within the budget by itself
        t = bh.bh_submit(ctx, tables, bh.make_view(v), None)
        out = torch.zeros((16, 16, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t2 = bh.bh_submit(ctx, tables, bh.make_view(v), out.data_ptr())
        bh.bh_serve_drain(ctx)
        with pytest.raises(bh.BhError) as ei:
            bh.bh_poll(ctx, t)
        assert ei.value.status == bh.BH_ENOMEM
        assert bh.bh_poll(ctx, t2)[0]
        bh.bh_ticket_free(ctx, t)
        bh.bh_ticket_free(ctx, t2)
        assert np.isfinite(out.cpu().numpy()).all()
    finally:
        bh.bh_destroy(ctx)


def test_batched_views_sampled_parity(gpu_ctx, gpu_tables, orc, orc_tables, big_field_scene):
    """Eight of the 64 uneven batch views (cameras from r = 2.5 to 50 moving at up to 0.95c
    in random directions, random disc radii and inclinations), rendered in one batched
    launch with the 1M-star map: a seeded 1% of each frame's quads against the oracle."""
    import torch
    field, n0, h, cube = big_field_scene
    views = scenes.batch_views(64, 3)
    pick = [0, 5, 11, 23, 31, 40, 52, 63]
    sel = [views[k] for k in pick]
    outs = [torch.zeros((v.height, v.width, 4), dtype=torch.float32, device="cuda") for v in sel]
    bh.bh_render_batch(gpu_ctx, gpu_tables, [bh.make_view(v, h) for v in sel],
                       [o.data_ptr() for o in outs], bh.current_stream())
    torch.cuda.synchronize()
    worst = {}
    for k, v, o in zip(pick, sel, outs):
        rgb = o.cpu().numpy()
        _, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h)     # AOV of the same frame
        quads = scenes.sample_quads(v.width, v.height, 0.01, 100 + k)
        pt = orc.render_quads(v, quads, cube=cube, n0=n0, tables=orc_tables)
        g = parity.gpu_at(rgb, aov, pt)
        s = parity.compare(pt, g, "table")
        worst[k] = {"masked": s["masked_fraction"], "dprime_max": s["dprime_max"],
                    "disc_1e-3": parity.frac_within(pt, g, 1e-3, "disc"),
                    "star_2e-2": parity.frac_within(pt, g, 2e-2, "star"),
                    "speed": float(np.linalg.norm(v.cam_vel)),
                    "r": float(np.linalg.norm(v.cam_pos))}
        worst[k].update({"star_n": s["star_n"], "star_p99": s["star_rel_p99"],
                         "star_p50": s["star_rel_p50"], "disc_n": s["disc_n"],
                         "star_5e-2": parity.frac_within(pt, g, 5e-2, "star"),
                         "finite": bool(np.isfinite(rgb).all())})
    _report({"batch_views": worst})
    for k, w in worst.items():
        assert w["finite"]
        assert w["masked"] < 0.03
        assert w["dprime_max"] < 1e-3
        assert w["disc_1e-3"] > 0.99
        assert w["star_5e-2"] > 0.99
    # star pixels of all eight frames together (some frames sample only ~150 of them)
    n = sum(w["star_n"] for w in worst.values())
    within = sum(w["star_2e-2"] * w["star_n"] for w in worst.values())
    assert within / n > 0.99


def test_autotune_sweep_renders_every_form_bitwise_equal():
    """bh_autotune renders the views with every tile configuration in both batched forms
    (one workgroup per tile, then persistent workgroups on an atomic counter), the last
    being the persistent form of the last configuration, into the caller's images: those
    images, and a batch rendered afterwards with the chosen form, equal bh_render bit for
    bit.  A context of its own, so the choice does not carry into other tests."""
    import torch
    ctx = bh.bh_create(0, 0)
    try:
        tables = bh.bh_precompute_tables(ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        hs = gpu_star_map(ctx, scenes.star_field(20000, 0), 256, bh.BH_TEXEL_FP16)
        sizes = [(64, 48), (100, 37), (16, 16), (130, 66)]
        views = []
        for k, (w, h) in enumerate(sizes):
            v = scenes.small_static_view()
            v.width, v.height = w, h
            v.cam_pos = tuple(float(x) for x in
                              scenes.spherical_position(12.0 + 3 * k, math.radians(70 + 5 * k), 0.3 * k))
            v.cam_rot = scenes.look_rotation(-np.array(v.cam_pos))
            views.append(v)
        recs = [bh.make_view(v, hs) for v in views]
        outs = [torch.full((h, w, 4), float("nan"), dtype=torch.float32, device="cuda")
                for (w, h) in sizes]
        best, ms = bh.bh_autotune(ctx, tables, recs, [o.data_ptr() for o in outs], reps=1)
        torch.cuda.synchronize()
        assert 0 <= best < 2 * bh.bh_tile_config_count() and all(m > 0 for m in ms)
        swept = [o.cpu().numpy() for o in outs]
        for o in outs:
            o.fill_(float("nan"))
        bh.bh_render_batch(ctx, tables, recs, [o.data_ptr() for o in outs], bh.current_stream())
        torch.cuda.synchronize()
        chosen = [o.cpu().numpy() for o in outs]
        for (w, h), rec, a, b in zip(sizes, recs, swept, chosen):
            ref = torch.full((h, w, 4), float("nan"), dtype=torch.float32, device="cuda")
            bh.bh_render(ctx, tables, rec, ref.data_ptr(), None, bh.current_stream())
            torch.cuda.synchronize()
            r = ref.cpu().numpy()
            assert np.isfinite(r).all()
            assert np.array_equal(a, r) and np.array_equal(b, r)
    finally:
        bh.bh_destroy(ctx)


def test_batch_after_tables_are_replaced_matches_plain():
    """A captured batch launch holds the table pointers and sizes by value.  Releasing a
    table set and precomputing one of another size (whose arrays may reuse the freed
    addresses) must not replay the old launch: the second batch equals bh_render with the
    new tables bit for bit."""
    import torch
    ctx = bh.bh_create(0, 0)
    try:
        hs = gpu_star_map(ctx, scenes.star_field(20000, 0), 256, bh.BH_TEXEL_FP16)
        views = []
        for k, (w, h) in enumerate([(64, 48), (40, 72)]):
            v = scenes.small_static_view()
            v.width, v.height = w, h
            views.append(bh.make_view(v, hs))
        outs = [torch.empty((v.height, v.width, 4), dtype=torch.float32, device="cuda")
                for v in views]
        ptrs = [o.data_ptr() for o in outs]
        st = bh.current_stream()
        for d_n, u_ne, u_nphi in ((512, 64, 32), (512, 128, 64), (256, 64, 32)):
            t = bh.bh_precompute_tables(ctx, d_n, u_ne, u_nphi, bh.BH_TAB_FP64_BAND, 0.05)
            bh.bh_render_batch(ctx, t, views, ptrs, st)
            torch.cuda.synchronize()
            got = [o.cpu().numpy().copy() for o in outs]
            for v, o, g in zip(views, outs, got):
                o.zero_()
                bh.bh_render(ctx, t, v, o.data_ptr(), None, st)
                torch.cuda.synchronize()
                assert np.array_equal(o.cpu().numpy(), g), (d_n, u_ne, u_nphi)
            bh.bh_release_tables(t)
        bh.bh_release_stars(hs)
    finally:
        bh.bh_destroy(ctx)
