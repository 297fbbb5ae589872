"""GPU (libbh, HIP gfx950) against the FP64 oracle, through the C ABI.

Tolerances.  Geometry: the paper's TraceRay bound is 1e-3 (Section 4); against the oracle's
own quadrature tables (same method, FP64) the FP32 path must be far tighter.  Colours are
compared per pixel relative to the pixel's brightest band, on pixels outside the mask
described in tests/parity.py; the masked fraction is reported and bounded."""
import json
import math

import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

from conftest import gpu_star_map
import parity

pytestmark = pytest.mark.gpu


def _report(s):
    print("\nPARITY " + json.dumps(s, sort_keys=True))


def test_tables_match_quadrature(gpu_ctx, gpu_tables, orc_tables):
    """Deflection and intersection tables integrated on the GPU (RK4, FP64 band) against
    quadrature at the same texel centres."""
    import torch
    D = np.zeros((512, 512), np.float32)
    U = np.zeros((32, 64), np.float32)
    bh.bh_tables_download(gpu_tables, D.ctypes.data, U.ctypes.data)
    oD, oU = orc_tables.D, orc_tables.U
    errD = np.abs(D - oD) / np.maximum(1.0, np.abs(oD))
    errU = np.abs(U - oU)
    s = {"D_max": float(errD.max()), "D_left_max": float(errD[:, :256].max()),
         "D_right_max": float(errD[:, 256:].max()), "D_p99": float(np.percentile(errD, 99)),
         "U_max": float(errU.max()), "worst_D_at": [int(v) for v in np.unravel_index(errD.argmax(), errD.shape)]}
    _report(s)
    assert np.isfinite(D).all() and np.isfinite(U).all()
    assert s["D_max"] < 1e-6
    assert s["U_max"] < 1e-6


def test_band_table_matches_quadrature(gpu_ctx, orc):
    import torch
    rng = np.random.default_rng(3)
    T = 10 ** rng.uniform(math.log10(300), math.log10(3e5), 2000)
    t = torch.from_numpy(T.astype(np.float32)).cuda()
    out = torch.zeros((len(T), 3), dtype=torch.float32, device="cuda")
    bh.bh_band_eval(gpu_ctx, t.data_ptr(), len(T), out.data_ptr(), bh.current_stream())
    torch.cuda.synchronize()
    g = out.cpu().numpy().astype(np.float64)
    ref = np.array([orc.band_radiance(float(x)) for x in t.cpu().numpy()])
    rel = np.abs(g - ref) / ref
    _report({"band_rel_max": float(rel.max()), "band_rel_p99": float(np.percentile(rel, 99))})
    assert rel.max() < 1e-3


@pytest.mark.parametrize("fmt", [bh.BH_TEXEL_FP16, bh.BH_TEXEL_FP32])
def test_star_map_matches_oracle(gpu_ctx, orc, fmt):
    field = scenes.star_field(20000, 0)
    n0 = 256
    h = gpu_star_map(gpu_ctx, field, n0, fmt)
    ref = orc.cubemap(field, n0)
    stats = {}
    for L in (0, 2, 5, 8):
        nl = n0 >> L
        g = np.zeros((6, nl, nl, 4), np.float32)
        bh.bh_stars_download(h, L, g.ctypes.data)
        o = orc.cubemap_level(ref, n0, L)
        occ_o, occ_g = o[..., 0] > 0, g[..., 0] > 0
        both = occ_o & occ_g
        relI = np.abs(g[..., 0][both] - o[..., 0][both]) / o[..., 0][both]
        relT = np.abs(g[..., 1][both] - o[..., 1][both]) / o[..., 1][both]
        dpos = np.abs(g[..., 2:][both] - o[..., 2:][both])
        stats[L] = {"occ_mismatch": int((occ_o != occ_g).sum()), "occupied": int(occ_o.sum()),
                    "I_rel": float(relI.max()), "T_rel": float(relT.max()),
                    "pos": float(dpos.max())}
        tol = 2e-3 if fmt == bh.BH_TEXEL_FP16 else 2e-5
        assert stats[L]["occ_mismatch"] <= max(2, occ_o.sum() // 2000)
        assert np.percentile(relI, 99.9) < tol and np.percentile(relT, 99.9) < tol
    _report({"fmt": fmt, "levels": stats})
    bh.bh_release_stars(h)


def _random_rays(n, seed):
    rng = np.random.default_rng(seed)
    u = 1 / rng.uniform(2.5, 50, n)
    d = rng.uniform(0.01, math.pi - 0.01, n)
    a = rng.uniform(0, math.pi, n)
    ric = rng.uniform(3, 6, n)
    roc = rng.uniform(10, 30, n)
    return np.stack([u, d, a, 1 / ric, 1 / roc], axis=1).astype(np.float32)


def test_traceray_matches_oracle(gpu_ctx, gpu_tables, orc, orc_tables):
    """TraceRay alone (Algorithm 1) in FP32 on the GPU against the oracle's FP64 TraceRay on
    quadrature tables (same method) and against exact integration (the paper's test)."""
    import torch
    rays = _random_rays(20000, 9)
    r = torch.from_numpy(rays).cuda()
    out = torch.zeros((len(rays), 4), dtype=torch.float32, device="cuda")
    bh.bh_trace_rays(gpu_ctx, gpu_tables, r.data_ptr(), len(rays), out.data_ptr(),
                     bh.current_stream())
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    bits = g[:, 3].copy().view(np.uint32)
    stats = {}
    for mode in ("table", "exact"):
        agree = n = agree_all = n_all = 0
        dmax = umax = 0.0
        for k in range(len(rays)):
            u, d, a, uic, uoc = [float(x) for x in rays[k]]
            e2 = (u / math.tan(d)) ** 2 + u * u * (1 - u)
            if abs(e2 / orc.MU - 1) < 1e-3:
                continue
            o = orc_tables.trace(u, d, a, uic, uoc) if mode == "table" else \
                orc.trace_exact(u, d, a, uic, uoc)
            cap = bool(bits[k] & 1)
            nc = int((bits[k] >> 1) & 1) + int((bits[k] >> 2) & 1)
            same = cap == o["captured"] and nc == o["n_cross"]
            n_all += 1
            agree_all += same
            # the 64-column intersection table interpolates toward its e = 0 column below
            # e ~ 0.08, where the method itself (also in FP64) misplaces crossings
            if e2 >= 0.08 ** 2:
                n += 1
                agree += same
            if not same or (e2 < 0.08 ** 2 and nc):
                continue
            if not cap:
                dmax = max(dmax, abs(o["delta_prime"] - g[k, 0]))
            for j in range(nc):
                umax = max(umax, abs(o["u"][j] - g[k, 1 + j]))
        stats[mode] = {"n": n, "agree": agree / n, "agree_all_e": agree_all / n_all,
                       "dprime_max": float(dmax), "u_max": float(umax)}
    _report(stats)
    assert stats["table"]["agree_all_e"] > 0.998
    assert stats["table"]["dprime_max"] < 5e-4 and stats["table"]["u_max"] < 2e-4
    assert stats["exact"]["agree"] > 0.995
    assert stats["exact"]["dprime_max"] < 1e-3 and stats["exact"]["u_max"] < 1e-3


def test_small_static_view_full_frame(gpu_ctx, gpu_tables, orc, orc_tables, small_scene):
    """128x128 static camera at r = 15: every pixel against the oracle."""
    field, n0, h, cube = small_scene
    v = scenes.small_static_view()
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    assert np.all(rgb[..., 3] == 1.0)
    quads = scenes.all_quads(v.width, v.height)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    pt = orc.render_quads(v, quads, cube=cube, n0=n0, tables=orc_tables)
    g = parity.gpu_at(rgb, aov, pe)
    se, st = parity.compare(pe, g, "exact"), parity.compare(pt, g, "table")
    _report({"small_exact": se, "small_table": st})
    assert se["finite"]
    assert se["masked_fraction"] < 0.02 and st["masked_fraction"] < 0.02
    # same method in FP64 (quadrature tables + TraceRay): FP32 trace, FP16 star map
    assert st["dprime_max"] < 5e-4 and st["u_max"] < 2e-4
    assert parity.frac_within(pt, g, 1e-3, "disc") > 0.995
    assert parity.frac_within(pt, g, 2e-2, "star") > 0.99
    assert parity.frac_within(pt, g, 2e-2, "all") > 0.995
    # exact geodesics: the method's own accuracy (paper bound 1e-3 on delta' and u); star
    # pixels also see sub-pixel star displacements from the table's delta' error, so the GPU
    # must match what the method itself reaches: the oracle's own table mode against exact
    # mode, with the same masks, within one percentage point
    assert se["dprime_max"] < 1e-3 and se["u_max"] < 1e-3
    meth = parity.frac_within(pe, parity.oracle_as_gpu(pt), 3e-2, "star")
    _report({"small_star_within_3e-2": {"gpu": parity.frac_within(pe, g, 3e-2, "star"),
                                        "oracle_tables": meth}})
    assert parity.frac_within(pe, g, 5e-2, "disc") > 0.99
    assert parity.frac_within(pe, g, 3e-2, "star") > min(0.97, meth - 0.01)
    assert parity.frac_within(pe, g, 3e-2, "all") > 0.99


def test_boosted_orbit_view_sampled(gpu_ctx, gpu_tables, orc, orc_tables, big_field_scene):
    """1920x1080 camera at r = 6 moving at 0.9c: a seeded 1% of the quads."""
    field, n0, h, cube = big_field_scene
    v = scenes.boosted_orbit_view()
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    quads = scenes.sample_quads(v.width, v.height, 0.01, 12)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    pt = orc.render_quads(v, quads, cube=cube, n0=n0, tables=orc_tables)
    g = parity.gpu_at(rgb, aov, pe)
    se, st = parity.compare(pe, g, "exact"), parity.compare(pt, g, "table")
    _report({"boosted_exact": se, "boosted_table": st})
    assert np.isfinite(rgb).all()
    assert se["masked_fraction"] < 0.02 and st["masked_fraction"] < 0.02
    assert st["dprime_max"] < 1e-3 and st["dprime_p99"] < 1e-5 and st["u_max"] < 2e-4
    assert parity.frac_within(pt, g, 1e-3, "disc") > 0.995
    assert parity.frac_within(pt, g, 2e-2, "star") > 0.99
    assert parity.frac_within(pt, g, 2e-2, "all") > 0.995
    assert se["dprime_max"] < 1e-3 and se["u_max"] < 1e-3
    # Exact mode: at 1080p a pixel is 1e-3 rad, and the tables' delta' error (p99 4e-5 rad
    # on these star pixels) moves gathered stars by a few hundredths of a pixel, magnified
    # near the shadow where Omega/Omega' is large.  The oracle's own table mode therefore
    # keeps only about 95% of star pixels within 3e-2 of exact mode (p99 0.10), and that is
    # the bar: the GPU must reach the method's own fraction within one percentage point.
    meth = parity.frac_within(pe, parity.oracle_as_gpu(pt), 3e-2, "star")
    gpu = parity.frac_within(pe, g, 3e-2, "star")
    _report({"boosted_star_within_3e-2": {"gpu": gpu, "oracle_tables": meth}})
    assert parity.frac_within(pe, g, 5e-2, "disc") > 0.99
    assert gpu > meth - 0.01 and meth > 0.9
    assert parity.frac_within(pe, g, 3e-2, "all") > 0.98


def test_batch_is_bitwise_equal_to_plain(gpu_ctx, gpu_tables, small_scene):
    import torch
    field, n0, h, cube = small_scene
    views = [v for v in scenes.batch_views(64, 3) if v.width * v.height <= 1024 * 1024][:6]
    outs = [torch.zeros((v.height, v.width, 4), dtype=torch.float32, device="cuda") for v in views]
    bh.bh_render_batch(gpu_ctx, gpu_tables, [bh.make_view(v, h) for v in views],
                       [o.data_ptr() for o in outs], bh.current_stream())
    torch.cuda.synchronize()
    for v, o in zip(views, outs):
        ref, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, h, aov=False)
        assert np.array_equal(o.cpu().numpy(), ref)


def test_serving_is_bitwise_equal_to_plain(gpu_ctx, gpu_tables, small_scene):
    import torch
    field, n0, h, cube = small_scene
    ctx = bh.bh_create(0, 0)
    try:
        bh.bh_serve_start(ctx, 0, 2, 64)   # small launches: frames are split and mixed
        views = scenes.batch_views(8, 5)
        outs = [torch.zeros((v.height, v.width, 4), dtype=torch.float32, device="cuda")
                for v in views]
        torch.cuda.synchronize()
        tickets = [bh.bh_submit(ctx, gpu_tables, bh.make_view(v, h), o.data_ptr())
                   for v, o in zip(views, outs)]
        bh.bh_serve_drain(ctx)
        for t in tickets:
            done, lat = bh.bh_poll(ctx, t)
            assert done and lat > 0
        for v, o in zip(views, outs):
            ref, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, h, aov=False)
            assert np.array_equal(o.cpu().numpy(), ref)
    finally:
        bh.bh_destroy(ctx)


def test_invalid_views_are_rejected(gpu_ctx, gpu_tables):
    import torch
    out = torch.zeros((8, 8, 4), dtype=torch.float32, device="cuda")
    base = scenes.small_static_view()
    bad = []
    for field, value in (("cam_pos", (0.5, 0.0, 0.0)), ("cam_vel", (0.0, 1.0, 0.0)),
                         ("disc_r_in", 2.5), ("fov_y", 0.0), ("r_s", -1.0),
                         ("disc_T0", float("nan"))):
        v = scenes.View(**{**base.__dict__, "width": 8, "height": 8, field: value})
        bad.append(v)
    for v in bad:
        with pytest.raises(bh.BhError) as ei:
            bh.bh_render(gpu_ctx, gpu_tables, bh.make_view(v), out.data_ptr())
        assert ei.value.status == bh.BH_EINVAL
