"""Pins of the oracle's bloom (Section 3.4.3: small-support filters on the mipmaps of the
final image approximate a point spread function).

Expected values come from properties any such filter bank must have (a constant image
stays constant, a linear image is reproduced away from the edges, an interior impulse keeps
its flux), from an independent 1D model of one level (the 2D filter is separable, so an
impulse's response is the outer product of 1D responses built here with numpy), and from a
hand-computed 2 x 2 example."""
import numpy as np
import pytest


def _weights(levels, seed=0):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 1.0, levels + 1)
    return w / w.sum()


@pytest.mark.parametrize("shape,levels", [((37, 53), 4), ((64, 64), 6), ((1, 9), 3),
                                          ((5, 1), 2), ((1, 1), 5)])
def test_constant_image_stays_constant(orc, shape, levels):
    img = np.empty(shape + (4,))
    img[...] = [0.3, 2.0, 7.0, 1.0]
    w = _weights(levels, 1)
    out = orc.bloom(img, levels, w)
    assert np.allclose(out, img, rtol=1e-14, atol=0)


def test_linear_image_is_reproduced_in_the_interior(orc):
    """Box averages of a linear function are the function at the coarse pixel centres,
    and bilinear interpolation reproduces linear functions, so with weights summing to 1
    the output equals the input wherever no clamp is involved."""
    h, w, L = 96, 128, 3
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    img = np.stack([0.5 + 0.01 * x, 2.0 - 0.02 * y, 0.003 * x + 0.004 * y, np.ones_like(x)], -1)
    out = orc.bloom(img, L, _weights(L, 2))
    m = 2 ** (L + 2)  # margin beyond which edge clamping cannot reach
    assert np.allclose(out[m:-m, m:-m], img[m:-m, m:-m], rtol=1e-13, atol=1e-13)
    assert not np.allclose(out[:2], img[:2], atol=1e-6)  # the clamp does change the edge


def test_interior_impulse_keeps_its_flux(orc):
    L = 5
    img = np.zeros((256, 256, 4))
    img[130, 101] = [1.0, 2.0, 3.0, 4.0]
    w = _weights(L, 3)
    out = orc.bloom(img, L, w)
    assert np.allclose(out.sum(axis=(0, 1)), [1.0, 2.0, 3.0, 4.0], rtol=1e-13)
    # and the response spreads: the impulse pixel keeps less than w_0 + the coarse share
    assert out[130, 101, 0] < 1.0


def _down1(v):
    n2 = (len(v) + 1) // 2
    idx = np.minimum(np.arange(2 * n2), len(v) - 1)
    return 0.5 * (v[idx[0::2]] + v[idx[1::2]])


def _up1(c, n):
    """Bilinear doubling: fine pixel x samples the coarse grid at x/2 - 1/4."""
    out = np.empty(n)
    for x in range(n):
        pos = x / 2.0 - 0.25
        i0 = int(np.floor(pos))
        f = pos - i0
        a, b = np.clip([i0, i0 + 1], 0, len(c) - 1)
        out[x] = (1 - f) * c[a] + f * c[b]
    return out


def _level_response_1d(n, x0, k):
    """1D response at full resolution of level k alone to a unit impulse at x0."""
    v = np.zeros(n)
    v[x0] = 1.0
    sizes = [n]
    for _ in range(k):
        v = _down1(v)
        sizes.append(len(v))
    for j in range(k, 0, -1):
        v = _up1(v, sizes[j - 1])
    return v


@pytest.mark.parametrize("k", [1, 2, 3])
def test_single_level_response_is_the_separable_1d_model(orc, k):
    h, w = 40, 57
    y0, x0 = 17, 30
    img = np.zeros((h, w, 4))
    img[y0, x0, 1] = 1.0
    wt = np.zeros(k + 1)
    wt[k] = 1.0
    out = orc.bloom(img, k, wt)[..., 1]
    want = np.outer(_level_response_1d(h, y0, k), _level_response_1d(w, x0, k))
    assert np.allclose(out, want, rtol=0, atol=1e-15)
    # near an edge too (the clamps of both models agree)
    img[...] = 0
    img[1, 0, 1] = 1.0
    out = orc.bloom(img, k, wt)[..., 1]
    want = np.outer(_level_response_1d(h, 1, k), _level_response_1d(w, 0, k))
    assert np.allclose(out, want, rtol=0, atol=1e-15)


def test_two_by_two_by_hand(orc):
    """One level over a 2 x 2 image [[a, b], [c, d]]: level 1 is the mean m; every output
    pixel is w0 * its own value + w1 * m (bilinear reads of a 1 x 1 level are m)."""
    img = np.zeros((2, 2, 4))
    img[..., 0] = [[1.0, 2.0], [3.0, 6.0]]
    out = orc.bloom(img, 1, [0.25, 0.75])[..., 0]
    assert np.allclose(out, 0.25 * img[..., 0] + 0.75 * 3.0, rtol=1e-15)


def test_no_levels_is_a_scale(orc):
    img = np.random.default_rng(4).uniform(0, 5, (7, 9, 4))
    assert np.array_equal(orc.bloom(img, 0, [0.5]), 0.5 * img)
