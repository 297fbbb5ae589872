/*
 * Display encoding of the final image: the tone mapping that follows the glare pass
 * (Section 3.4.3 applies glare before tone mapping).  TEST INFRASTRUCTURE ONLY (see
 * bh_oracle.h).
 *
 * The paper prints no tone mapping operator; this is its reading, per colour channel c of a
 * linear RGBA pixel, in plain FP64:
 *   x = exposure * c;
 *   y = 1 - exp(-x) for x > 0, else 0 (negative, zero and NaN inputs give 0);
 *   v = the sRGB transfer function of y (IEC 61966-2-1): 12.92 y for y <= 0.0031308,
 *       else 1.055 y^(1/2.4) - 0.055;
 *   code = floor(255 v + 1/2)  (v < 1, so code <= 255).
 * Alpha is encoded as 255.  Each pixel becomes 4 bytes R, G, B, A.
 */
#include <math.h>
#include <stdint.h>

#include "bh_oracle.h"

static double tone_curve(double x) { return x > 0.0 ? 1.0 - exp(-x) : 0.0; }

static double srgb_transfer(double y) {
  return y <= 0.0031308 ? 12.92 * y : 1.055 * pow(y, 1.0 / 2.4) - 0.055;
}

int orc_tonemap(const double* in, int64_t n, double exposure, uint8_t* out, double* scaled) {
  if (!in || !out || n < 0 || !(exposure > 0.0) || !isfinite(exposure)) return 1;
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) {
      const double s = 255.0 * srgb_transfer(tone_curve(exposure * in[4 * i + c])) + 0.5;
      out[4 * i + c] = (uint8_t)floor(s);
      if (scaled) scaled[3 * i + c] = s;
    }
    out[4 * i + 3] = 255;
  }
  return 0;
}
