"""Pins of the oracle's display encoding (tone curve 1 - exp(-x), sRGB transfer function,
8-bit codes), the tone mapping that follows the glare pass of Section 3.4.3.

The expected codes come from the inverse of each stage, written independently of the
oracle's forward formulas: the sRGB decoding function of IEC 61966-2-1 and the inverse tone
curve -log1p(-y).  Every one of the 255 code boundaries is located that way and the oracle
must step from code k - 1 to code k across it; a wrong exponent, constant, threshold,
rounding rule or tone curve moves the boundaries and fails.  Published sRGB values (18%
grey is code 118, half linear intensity is code 188, code 128 decodes to 0.2158605) are
checked on top."""
import math

import numpy as np
import pytest


def _decode(v):
    """sRGB decoding (IEC 61966-2-1): non-linear value v in [0, 1] to linear intensity."""
    return v / 12.92 if v <= 0.04045 else ((v + 0.055) / 1.055) ** 2.4


def _x_for_linear(y):
    """Input that the tone curve maps to linear display intensity y (exposure 1)."""
    return -math.log1p(-y)


def _codes(orc, xs, exposure=1.0):
    img = np.zeros((len(xs), 4))
    img[:, 0] = xs
    img[:, 1] = xs
    img[:, 2] = xs
    codes, scaled = orc.tonemap(img, exposure)
    assert np.all(codes[:, 0] == codes[:, 1]) and np.all(codes[:, 0] == codes[:, 2])
    return codes[:, 0].astype(int), codes[:, 3], scaled[:, 0]


def test_every_code_boundary_is_where_the_inverse_stages_put_it(orc):
    xs = []
    for k in range(1, 256):
        x = _x_for_linear(_decode((k - 0.5) / 255.0))
        xs += [x * (1.0 - 1e-9), x * (1.0 + 1e-9)]
    codes, alpha, scaled = _codes(orc, xs)
    assert np.all(codes[0::2] == np.arange(0, 255)) and np.all(codes[1::2] == np.arange(1, 256))
    # the value whose floor is the code sits next to the boundary k - 1/2 + 1/2 = k
    assert np.allclose(scaled[0::2], np.arange(1, 256), atol=1e-6)
    assert np.all(alpha == 255)


def test_published_srgb_values(orc):
    lin = [0.18, 0.5, 0.2158605, 0.0, 1.0 - 1e-12]
    codes, _, _ = _codes(orc, [_x_for_linear(y) for y in lin])
    assert list(codes) == [118, 188, 128, 0, 255]


def test_tone_curve_special_values(orc):
    codes, alpha, _ = _codes(orc, [math.log(2.0), 1e30, math.inf, 0.0, -1.0, -math.inf, math.nan])
    # ln 2 is half the display range, i.e. linear 1/2 (code 188); saturation gives 255;
    # zero, negative and NaN inputs give 0
    assert list(codes) == [188, 255, 255, 0, 0, 0, 0]
    assert np.all(alpha == 255)


def test_codes_rise_with_the_input_and_reach_every_value(orc):
    xs = np.concatenate([np.linspace(0.0, 1e-3, 4001), np.geomspace(1e-3, 60.0, 40000)])
    codes, _, _ = _codes(orc, xs)
    assert np.all(np.diff(codes) >= 0)
    assert set(codes.tolist()) == set(range(256))


def test_exposure_scales_the_input_and_channels_are_independent(orc):
    rng = np.random.default_rng(17)
    img = rng.uniform(0.0, 3.0, (50, 40, 4))
    a, _ = orc.tonemap(img, 0.37)
    b, _ = orc.tonemap(img * 0.37, 1.0)
    assert np.array_equal(a, b)
    perm = img[..., [2, 0, 1, 3]]
    c, _ = orc.tonemap(perm, 0.37)
    assert np.array_equal(c[..., :3], a[..., [2, 0, 1]])


@pytest.mark.parametrize("exposure", [0.0, -1.0, math.inf, math.nan])
def test_bad_exposure_is_rejected(orc, exposure):
    with pytest.raises(ValueError):
        orc.tonemap(np.zeros((2, 2, 4)), exposure)
