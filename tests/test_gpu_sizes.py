"""The largest frames: 7680x4320 (the biggest frame of the serving mix) and the 65536-pixel
limit on a side, against the oracle on seeded samples of quads (same tolerances and mask as
the 1080p parity test); sizes past the limits (65536 a side, 2^31 pixels or elements, batches
whose tiles hold 2^32 pixels) are refused."""
import json

import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

import parity

pytestmark = pytest.mark.gpu


def _report(s):
    print("\nPARITY " + json.dumps(s, sort_keys=True))


def test_8k_boosted_frame_sampled(gpu_ctx, gpu_tables, orc, orc_tables, big_field_scene):
    field, n0, h, cube = big_field_scene
    v = scenes.boosted_orbit_view(7680, 4320)
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    assert np.isfinite(rgb).all() and np.all(rgb[..., 3] == 1.0)
    quads = scenes.sample_quads(v.width, v.height, 0.0006, 31)
    pt = orc.render_quads(v, quads, cube=cube, n0=n0, tables=orc_tables)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    g = parity.gpu_at(rgb, aov, pt)
    st, se = parity.compare(pt, g, "table"), parity.compare(pe, g, "exact")
    _report({"8k_table": st, "8k_exact": se})
    assert st["masked_fraction"] < 0.02 and se["masked_fraction"] < 0.02
    assert st["dprime_max"] < 1e-3 and st["dprime_p99"] < 1e-5 and st["u_max"] < 2e-4
    assert parity.frac_within(pt, g, 1e-3, "disc") > 0.995
    # star light follows the beam's escape direction against the pixel grid: FP32 delta'
    # differs from table mode by 3e-6 rad at p99, 1.3% of an 8K pixel (2.4e-4 rad, four times
    # smaller than at 1080p), which moves tent weights by up to ~2.5%; hence 5e-2 here
    assert parity.frac_within(pt, g, 5e-2, "star") > 0.99
    assert se["dprime_max"] < 1e-3 and se["u_max"] < 1e-3
    assert parity.frac_within(pe, g, 5e-2, "disc") > 0.99


@pytest.mark.parametrize("W,H", [(65536, 2), (2, 65536), (65535, 3)])
def test_frames_at_the_size_limit(gpu_ctx, gpu_tables, orc, orc_tables, W, H):
    """One side at the 65536-pixel limit (and one pixel under it, odd): every pixel is
    written, and sampled quads agree with the oracle's table mode."""
    from conftest import gpu_star_map
    field = scenes.star_field(20000, 0)
    hs = gpu_star_map(gpu_ctx, field, 256, bh.BH_TEXEL_FP16)
    v = scenes.small_static_view()
    v.width, v.height = W, H
    rgb, aov = parity.render_gpu(gpu_ctx, gpu_tables, v, hs)
    assert rgb.shape == (H, W, 4) and np.isfinite(rgb).all() and np.all(rgb[..., 3] == 1.0)
    quads = scenes.sample_quads(W, H, 0.05, 32)
    quads = quads[(quads[:, 0] + 1 < W) & (quads[:, 1] + 1 < H)]  # whole quads only
    pt = orc.render_quads(v, quads, cube=orc.cubemap(field, 256), n0=256, tables=orc_tables)
    g = parity.gpu_at(rgb, aov, pt)
    st = parity.compare(pt, g, "table")
    _report({"size": [W, H], "table": st})
    assert st["finite"] and st["masked_fraction"] < 0.05
    assert st["dprime_max"] < 1e-3 and st["u_max"] < 2e-4
    assert parity.frac_within(pt, g, 2e-2, "all") > 0.99


def test_views_beyond_the_size_limit_are_rejected(gpu_ctx, gpu_tables):
    import torch
    out = torch.zeros((4,), dtype=torch.float32, device="cuda")
    for W, H in ((65537, 1), (1, 65537), (0, 4), (4, 0)):
        v = scenes.small_static_view()
        v.width, v.height = W, H
        with pytest.raises(bh.BhError) as ei:
            bh.bh_render(gpu_ctx, gpu_tables, bh.make_view(v), out.data_ptr())
        assert ei.value.status == bh.BH_EINVAL


def test_sizes_beyond_one_launch_are_rejected(gpu_ctx, gpu_tables):
    """One launch covers fewer than 2^32 work-items: images above 2^31 pixels, arrays above
    2^31 rays or temperatures and batches whose tiles hold 2^32 pixels are refused before any
    device work (the buffers passed are small and never touched)."""
    import torch
    out = torch.zeros((8, 8, 4), dtype=torch.float32, device="cuda")
    base = scenes.small_static_view()
    for w, h in ((65536, 65536), (65536, 32769), (32769, 65536)):
        v = scenes.View(**{**base.__dict__, "width": w, "height": h})
        with pytest.raises(bh.BhError) as ei:
            bh.bh_render(gpu_ctx, gpu_tables, bh.make_view(v), out.data_ptr())
        assert ei.value.status == bh.BH_EINVAL
        with pytest.raises(bh.BhError) as ei:
            bh.bh_tonemap(gpu_ctx, out.data_ptr(), out.data_ptr() + 1024, w, h, 1.0)
        assert ei.value.status == bh.BH_EINVAL
    half = scenes.View(**{**base.__dict__, "width": 65536, "height": 32768})
    with pytest.raises(bh.BhError) as ei:
        bh.bh_render_batch(gpu_ctx, gpu_tables, [bh.make_view(half)] * 2,
                           [out.data_ptr()] * 2)
    assert ei.value.status == bh.BH_EINVAL
    n = (1 << 31) + 1
    p = out.data_ptr()
    for call in (lambda: bh.bh_trace_rays(gpu_ctx, gpu_tables, p, n, p),
                 lambda: bh.bh_trace_rays_timed(gpu_ctx, gpu_tables, p, n, p, p),
                 lambda: bh.bh_march_rays(gpu_ctx, p, n, 64, p),
                 lambda: bh.bh_band_eval(gpu_ctx, p, n, p)):
        with pytest.raises(bh.BhError) as ei:
            call()
        assert ei.value.status == bh.BH_EINVAL
    torch.cuda.synchronize()
    assert not out.any()
