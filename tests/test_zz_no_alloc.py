"""bh_render_batch_noalloc (the batched render for callers that cannot allocate) against
bh_render_batch through the C ABI: the same bits, two calls in a row with the second one
smaller, in both launch forms and two tile configurations, and no library allocation."""
import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

from conftest import gpu_star_map

pytestmark = pytest.mark.gpu


def _views(sizes, stars, seed):
    rng = np.random.default_rng(seed)
    out = []
    for w, h in sizes:
        v = scenes.small_static_view()
        v.width, v.height = w, h
        v.fov_y = float(rng.uniform(0.6, 1.4))
        out.append(bh.make_view(v, stars))
    return out


def test_noalloc_batch_equals_batch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = bh.bh_create(0, 0)
    try:
        tables = bh.bh_precompute_tables(ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        stars = gpu_star_map(ctx, scenes.star_field(20000, 0), 256, bh.BH_TEXEL_FP16)
        st = bh.current_stream()
        calls = [_views([(96, 64), (40, 72), (130, 66), (16, 16), (64, 48)], stars, 1),
                 _views([(33, 17), (24, 40)], stars, 2)]
        for cfg in (0, 3):
            bh.bh_set_tile_config(ctx, cfg)
            for form in (0, 1):
                bh.bh_set_batch_form(ctx, form)
                for views in calls:
                    ref = [torch.full((v.height, v.width, 4), -1.0, device="cuda") for v in views]
                    got = [torch.full((v.height, v.width, 4), -2.0, device="cuda") for v in views]
                    bh.bh_render_batch(ctx, tables, views, [o.data_ptr() for o in ref], st)
                    torch.cuda.synchronize()
                    used = bh.bh_bytes_in_use(ctx)
                    bh.bh_render_batch_noalloc(ctx, tables, views, [o.data_ptr() for o in got], st)
                    torch.cuda.synchronize()
                    assert bh.bh_bytes_in_use(ctx) == used
                    for k, (r, g) in enumerate(zip(ref, got)):
                        assert torch.equal(r, g), (cfg, form, k)
                        assert bool(torch.isfinite(g).all())
        too_many = calls[1] * 257
        outs = [0] * len(too_many)
        with pytest.raises(bh.BhError) as e:
            bh.bh_render_batch_noalloc(ctx, tables, too_many, outs, st)
        assert e.value.status == bh.BH_EINVAL
        bh.bh_release_stars(stars)
        bh.bh_release_tables(tables)
    finally:
        bh.bh_destroy(ctx)
