"""Bloom (Section 3.4.3, mipmap filters approximating a point spread function) on the GPU,
through the C ABI, against the oracle's FP64 bloom.

Tolerance.  Each output value is a weighted sum of box averages and bilinear blends, every
term with non-negative weights; FP32 rounds each of the ~4 operations per level at 2^-24
relative, so |GPU - oracle| stays below ~K * 4 * 2^-24 of the largest contributing value.
The bound used is 2e-6 of the image's largest value (K <= 16 levels)."""
import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

pytestmark = pytest.mark.gpu


def _bloom_gpu(ctx, img, levels, weights, handle=None, in_place=False, stream=None):
    import torch
    h, w = img.shape[:2]
    t = torch.from_numpy(np.ascontiguousarray(img, np.float32)).cuda()
    out = t if in_place else torch.full_like(t, float("nan"))
    b = handle or bh.bh_bloom_create(ctx, w, h, levels)
    try:
        bh.bh_bloom_apply(b, weights, t.data_ptr(), out.data_ptr(),
                          stream if stream is not None else bh.current_stream())
        torch.cuda.synchronize()
    finally:
        if handle is None:
            bh.bh_bloom_release(b)
    return out.cpu().numpy()


# exactly 7 levels takes the output pass's own U_7 (no tail launch): ragged and tiny sizes
# of that depth are included
CASES = [(1, 1, 0), (1, 1, 3), (3, 5, 2), (64, 64, 6), (65, 33, 7), (130, 70, 9),
         (200, 129, 16), (64, 1, 8), (1, 300, 10), (257, 130, 7), (1920, 1080, 7),
         (3840, 2160, 8), (1, 1, 7), (3, 200, 7), (700, 5, 7)]


@pytest.mark.parametrize("w,h,levels", CASES)
def test_bloom_matches_the_oracle(gpu_ctx, orc, w, h, levels):
    rng = np.random.default_rng(w * 7919 + h * 31 + levels)
    img = rng.uniform(0.0, 1.0, (h, w, 4)).astype(np.float32)
    wt = scenes.bloom_weights(levels)
    g = _bloom_gpu(gpu_ctx, img, levels, wt)
    o = orc.bloom(img.astype(np.float64), levels, np.asarray(wt, np.float32).astype(np.float64))
    err = np.abs(g - o).max()
    print("\nBLOOM %dx%d K=%d max|err| %.3g" % (w, h, levels, err))
    assert np.isfinite(g).all()
    assert err <= 2e-6 * np.abs(o).max()


def test_bloom_with_a_coarse_tail_beyond_shared_memory(gpu_ctx, orc):
    """12288 x 4096 with 9 levels: levels 7-9 hold 96x32 + 48x16 + 24x8 pixels, more than
    the tail kernel keeps in LDS, so it runs on global memory."""
    w, h, levels = 12288, 4096, 9
    rng = np.random.default_rng(77)
    img = rng.uniform(0.0, 1.0, (h, w, 4)).astype(np.float32)
    wt = scenes.bloom_weights(levels)
    g = _bloom_gpu(gpu_ctx, img, levels, wt)
    o = orc.bloom(img.astype(np.float64), levels, np.asarray(wt, np.float32).astype(np.float64))
    assert np.abs(g - o).max() <= 2e-6 * np.abs(o).max()


def test_bloom_of_a_rendered_frame(gpu_ctx, gpu_tables, orc, big_field_scene):
    """The 1080p boosted-orbit frame (HDR: stars and disc over a black sky) through 7 levels;
    in place and out of place give the same bits, and so do two calls in a row on one
    handle."""
    import parity
    field, n0, hs, cube = big_field_scene
    v = scenes.boosted_orbit_view()
    rgb, _ = parity.render_gpu(gpu_ctx, gpu_tables, v, hs, aov=False)
    wt = scenes.bloom_weights(7)
    b = bh.bh_bloom_create(gpu_ctx, v.width, v.height, 7)
    try:
        g1 = _bloom_gpu(gpu_ctx, rgb, 7, wt, handle=b)
        g2 = _bloom_gpu(gpu_ctx, rgb, 7, wt, handle=b, in_place=True)
        g3 = _bloom_gpu(gpu_ctx, rgb, 7, wt, handle=b)
    finally:
        bh.bh_bloom_release(b)
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)
    o = orc.bloom(rgb.astype(np.float64), 7, np.asarray(wt, np.float32).astype(np.float64))
    assert np.abs(g1 - o).max() <= 2e-6 * np.abs(o).max()
    # flux is kept up to the edges' share
    assert abs(g1[..., :3].sum() / rgb[..., :3].sum() - 1.0) < 1e-2


def test_two_handles_on_two_streams(gpu_ctx):
    import torch
    rng = np.random.default_rng(5)
    imgs = [rng.uniform(0, 1, (300, 500, 4)).astype(np.float32) for _ in range(2)]
    wt = scenes.bloom_weights(9)
    ref = [_bloom_gpu(gpu_ctx, im, 9, wt) for im in imgs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    hs = [bh.bh_bloom_create(gpu_ctx, 500, 300, 9) for _ in range(2)]
    try:
        ins = [torch.from_numpy(im).cuda() for im in imgs]
        outs = [torch.empty_like(t) for t in ins]
        torch.cuda.synchronize()
        for _ in range(5):
            for k in range(2):
                bh.bh_bloom_apply(hs[k], wt, ins[k].data_ptr(), outs[k].data_ptr(),
                                  streams[k].cuda_stream)
        torch.cuda.synchronize()
        for k in range(2):
            assert np.array_equal(outs[k].cpu().numpy(), ref[k])
    finally:
        for b in hs:
            bh.bh_bloom_release(b)


def test_bloom_rejects_bad_arguments(gpu_ctx):
    import torch
    for w, h, k in ((0, 4, 2), (4, -1, 2), (70000, 4, 2), (4, 4, 17), (4, 4, -1)):
        with pytest.raises(bh.BhError) as ei:
            bh.bh_bloom_create(gpu_ctx, w, h, k)
        assert ei.value.status == bh.BH_EINVAL
    b = bh.bh_bloom_create(gpu_ctx, 4, 4, 2)
    t = torch.zeros((4, 4, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(bh.BhError) as ei:
        bh.bh_bloom_apply(b, [0.5, float("nan"), 0.5], t.data_ptr(), t.data_ptr())
    assert ei.value.status == bh.BH_EINVAL
    with pytest.raises(bh.BhError) as ei:
        bh.bh_bloom_apply(b, [0.5, 0.25, 0.25], None, t.data_ptr())
    assert ei.value.status == bh.BH_EINVAL
    bh.bh_bloom_release(b)
