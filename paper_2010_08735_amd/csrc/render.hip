// Per-pixel beam tracer (Sections 3.2-3.4) for gfx950.
//
// Thread layout: one wavefront covers an 8x8 pixel block; lane l handles quad l >> 2 of
// the block (4x4 quads) and pixel (l & 1, (l >> 1) & 1) inside the quad, so the 2x2 quad
// partners needed for screen-space derivatives are lanes l^1 (same row) and l^2 (same
// column) and are read with DPP quad permutations.  A workgroup tile is TW x TH pixels made of
// 8x8 blocks; each wave walks PPT blocks.  Pixels outside the image are computed (their
// rays are valid) but not stored, so every quad is complete.
//
// Steps per pixel:
//   beam init   camera direction n_C -> aberration into the static frame (eq. d) ->
//               coordinate direction d (e_r has length sqrt(1-u), eq. staticbasis) ->
//               ray plane e_x', e_y', e_z', angle delta, disc angle alpha (eqs. raybasis,
//               alpha)
//   TraceRay    Algorithm 1 with bilinear fetches of D(e,u), D(e,u_a) and U(e,phi)
//   disc        T' from the temperature law, Doppler factor g(k,l)/g(k',l') with the
//               Keplerian k' (eq. k_prime), band radiances of a blackbody at D T'
//               (Section 3.4.2), front-to-back composite
//   stars       fine quad differences of d' and of q, face Jacobian, mip
//               level such that the extended footprint spans at most 9x9 texels,
//               tent-weighted gather f(w) f(h), lensing factor Omega/Omega', one Doppler
//               shift per pixel.
#include "bh_dev.h"

namespace bh {

struct __align__(8) Half4r {
  _Float16 x, y, z, w;
};
struct __align__(16) Half8r {
  _Float16 v[8];
};
struct __align__(8) OccPair {  // two words of two consecutive occupancy rows (stars.hip)
  uint32_t a0, a1, b0, b1;      // row r word k, row r + 1 word k, row r word k + 1, row r + 1 word k + 1
};

// Stored texels are (I, T, p_u, p_v); the FP16 format keeps I / scale_L and T / 1024, and
// the caller applies both factors once to the footprint sums.  Band-colour maps store
// (R, G, B, p_u, p_v, 0, 0, 0), FP16 bands divided by scale_L.
enum { kTexIT16 = 0, kTexIT32 = 1, kTexBand16 = 2, kTexBand32 = 3 };

// Footprint of one pixel on one star-map level: texel columns x0 .. x0 + 8 and rows
// y0 .. y0 + ny at most, read from the occupancy bits into one 81-bit mask (bit 9 r + c for
// row y0 + r, column x0 + c; rows 0-6 in `lo`, rows 7-8 in `hi`), then one pass over the set
// bits.  A single loop over occupied texels keeps the lanes of a wave in step far better
// than a loop per row.  Adds the tent-weighted sums of I and I T, in stored units, to A, B
// (FMT kTexIT16, kTexIT32), or of R, G, B to A, B, C (kTexBand16, kTexBand32).
struct Footprint {
  uint32_t texel0;       // texel index of (x0, y0)
  const uint32_t* occ;   // occupancy word of (x0, y0) in the row pair starting at y0
  int nL, wpr4, sh, ny;  // wpr4: occupancy words from one row pair to the pair two rows down
  uint32_t span;         // bit mask of the footprint's columns, shifted to bit 0
  // screen-space coordinates (w, h) of a star at (c + p_u, r + p_v) texels from the
  // footprint's corner: w = W0 + Wc (c + p_u) + Wr (r + p_v), h = H0 + Hc (..) + Hr (..)
  float W0, Wc, Wr, H0, Hc, Hr;
  float one;             // 1, not known to the compiler: p_u + c stays one mixed-precision FMA
};

// Buffers of the measurement variant (COUNT): one bit per star-map texel the footprints
// visit, and the total of the bytes every pixel requests through the caches (table and band
// table fetches, occupancy words, texels, level records, image and AOV stores).
struct CountBufs {
  uint32_t* touched;
  unsigned long long* l2_bytes;
};

template <int FMT, bool COUNT, bool PAIR = true>
__device__ __forceinline__ void gather(const void* tex, const Footprint& F, const CountBufs* cnt,
                                       uint32_t& req, float& A, float& B, float& C) {
  uint32_t w0 = 0, w1 = 0, hi = 0;  // lo = w0 + 2^32 w1
  // Every row's two occupancy words are loaded before any is used, so a lane waits once for
  // its rows instead of once per row.  Rows come in pairs (r, r + 1), one 16-byte load each
  // (the occupancy layout of stars.hip); pairs past the footprint load nothing, and the
  // second row of the last pair is dropped when it lies past the footprint.
  uint32_t ra[10], rb[10];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    ra[2 * p] = rb[2 * p] = ra[2 * p + 1] = rb[2 * p + 1] = 0u;
    if (2 * p <= F.ny) {
      const OccPair q = *(const OccPair*)(F.occ + (uint32_t)p * (uint32_t)F.wpr4);
      ra[2 * p] = q.a0;
      ra[2 * p + 1] = q.a1;
      rb[2 * p] = q.b0;
      rb[2 * p + 1] = q.b1;
    }
  }
  if (COUNT) req += 16 * (F.ny / 2 + 1);  // one 16-byte load per row pair
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    // the row's 9 columns from bit x0 & 31 of two consecutive words (a funnel shift)
    uint32_t b = __builtin_amdgcn_alignbit(rb[r], ra[r], (uint32_t)F.sh) & F.span;
    if ((r & 1) && r > F.ny) b = 0u;
    if (r < 3) {
      w0 |= b << (9 * r);
    } else if (r == 3) {
      w0 |= b << 27;
      w1 |= b >> 5;
    } else if (r < 7) {
      w1 |= b << (9 * r - 32);
    } else {
      hi |= b << (9 * (r - 7));
    }
  }
  uint64_t lo = (uint64_t)w0 | ((uint64_t)w1 << 32);
  // texels from the footprint's corner: row r, column c lies r nL + c = idx + r (nL - 9)
  // texels on (nL - 9 >= -8: a signed 24-bit product)
  const Half4r* tex16 = (const Half4r*)tex + F.texel0;
  const float4* tex32 = (const float4*)tex + F.texel0;
  const Half8r* texb16 = (const Half8r*)tex + F.texel0;
  const float4* texb32 = (const float4*)tex + 2 * (size_t)F.texel0;
  const int nLm9 = F.nL - 9;
  // the texel of mask bit idx (row r, column c lies r nL + c = idx + r (nL - 9) texels from
  // the footprint's corner)
  auto at = [&](int idx) {
    const int r = (idx * 57) >> 9;  // idx / 9 for idx < 81
    return (uint32_t)(__mul24(r, nLm9) + idx);
  };
  struct Tx {  // one stored texel of any format
    Half4r h4;
    Half8r h8;
    float4 f0, f1;
  };
  auto load = [&](uint32_t t) {
    Tx x;
    if constexpr (FMT == kTexIT16) x.h4 = tex16[t];
    if constexpr (FMT == kTexIT32) x.f0 = tex32[t];
    if constexpr (FMT == kTexBand16) x.h8 = texb16[t];
    if constexpr (FMT == kTexBand32) {
      x.f0 = texb32[2 * t];
      x.f1 = texb32[2 * t + 1];
    }
    return x;
  };
  // tent weight f(w) f(h) of the star of texel x at bit idx, 0 unless `use`, then the sums
  auto weigh = [&](const Tx& x, int idx, bool use) {
    const int r = (idx * 57) >> 9, c = idx - 9 * r;
    const float fc = (float)c, fr = (float)r;
    float a, b;
    if constexpr (FMT == kTexIT16) {
      // half operands go straight into mixed-precision multiply-adds
      a = fmaf((float)x.h4.z, F.one, fc);
      b = fmaf((float)x.h4.w, F.one, fr);
    } else if constexpr (FMT == kTexIT32) {
      a = fc + x.f0.z;
      b = fr + x.f0.w;
    } else if constexpr (FMT == kTexBand16) {
      a = fmaf((float)x.h8.v[3], F.one, fc);
      b = fmaf((float)x.h8.v[4], F.one, fr);
    } else {
      a = fc + x.f0.w;
      b = fr + x.f1.x;
    }
    const float w = fmaf(F.Wc, a, fmaf(F.Wr, b, F.W0));
    const float h = fmaf(F.Hc, a, fmaf(F.Hr, b, F.H0));
    float wt = __builtin_amdgcn_fmed3f(1.0f - fabsf(w), 0.0f, 1.0f) *
               __builtin_amdgcn_fmed3f(1.0f - fabsf(h), 0.0f, 1.0f);  // max(1 - |x|, 0)
    wt = use ? wt : 0.0f;
    if constexpr (FMT == kTexIT16) {
      const float wi = fmaf(wt, (float)x.h4.x, 0.0f);
      A += wi;
      B = fmaf(wi, (float)x.h4.y, B);
    } else if constexpr (FMT == kTexIT32) {
      const float wi = wt * x.f0.x;
      A += wi;
      B = fmaf(wi, x.f0.y, B);
    } else if constexpr (FMT == kTexBand16) {
      A = fmaf(wt, (float)x.h8.v[0], A);
      B = fmaf(wt, (float)x.h8.v[1], B);
      C = fmaf(wt, (float)x.h8.v[2], C);
    } else {
      A = fmaf(wt, x.f0.x, A);
      B = fmaf(wt, x.f0.y, B);
      C = fmaf(wt, x.f0.z, C);
    }
  };
  // Two taps per iteration, both texel loads in flight before either is weighed, so a lane
  // waits on its scattered loads half as often.  With one tap left the second repeats the
  // first texel with weight 0 and adds nothing: the sums take the taps in bit order.  Only
  // the bit indices stay live across the loads (row and column are recomputed after).
  auto two_taps = [&](int i0, int i1, bool two) {
    if (COUNT) {
      for (int k = 0; k < 2; ++k) {
        if (k == 1 && !two) break;
        const uint32_t ta = F.texel0 + at(k == 0 ? i0 : i1);
        atomicOr(&cnt->touched[ta >> 5], 1u << (ta & 31));
        req += FMT == kTexIT16 ? 8 : (FMT == kTexBand32 ? 32 : 16);
      }
    }
    const Tx x0 = load(at(i0)), x1 = load(at(i1));
    weigh(x0, i0, true);
    weigh(x1, i1, two);
  };
  if constexpr (PAIR && (FMT == kTexIT16 || FMT == kTexIT32)) {
    while (lo) {
      const int i0 = __builtin_ctzll(lo);
      lo &= lo - 1u;
      const bool two = lo != 0;
      const int i1 = two ? __builtin_ctzll(lo) : i0;
      lo &= lo - 1u;  // 0 stays 0
      two_taps(i0, i1, two);
    }
    while (hi) {
      const int i0 = 63 + __builtin_ctz(hi);
      hi &= hi - 1u;
      const bool two = hi != 0;
      const int i1 = two ? 63 + __builtin_ctz(hi) : i0;
      hi &= hi - 1u;
      two_taps(i0, i1, two);
    }
  } else {
    // band texels are twice as wide: one tap per iteration keeps the band kernels' register
    // budget (two in flight spilled 19 registers at 8 waves per SIMD), and the kernel for
    // band star maps without area maps takes (I, T) maps one tap at a time too (PAIR)
    auto one_tap = [&](int i) {
      if (COUNT) {
        const uint32_t ta = F.texel0 + at(i);
        atomicOr(&cnt->touched[ta >> 5], 1u << (ta & 31));
        req += FMT == kTexBand32 ? 32 : 16;
      }
      weigh(load(at(i)), i, true);
    };
    while (lo) {
      const int i = __builtin_ctzll(lo);
      lo &= lo - 1u;
      one_tap(i);
    }
    while (hi) {
      const int i = 63 + __builtin_ctz(hi);
      hi &= hi - 1u;
      one_tap(i);
    }
  }
}

struct TraceOut {
  float e;             // the beam's invariant e = sqrt(e^2)
  float dprime;        // escape angle (valid if !captured)
  float ucr[2];
  float tret[2];       // retarded times of the crossings (TIMED only)
  int mcr[2];          // crossing k lies at beam-plane angle alpha + mcr[k] pi (TIMED only)
  int ncross;
  unsigned bits;
  uint32_t req;        // bytes the table fetches request (read by the measurement variant only)
};

// singular part of the coordinate time along a ray: t = tau + S(u) + const
__device__ __forceinline__ float time_singular(float u) {
  return __log2f(fdiv(u, 1.0f - u)) * 0.693147180559945309f - fdiv(1.0f, u);
}

// Algorithm 1, TraceRay, in FP32.  Returns crossings in order along the beam.  TIMED also
// returns each crossing's retarded time (the coordinate time the light takes from it to
// the camera): s (t_0 - t) for crossing 0 and 2 t_a - t - t_1 for crossing 1, with
// t = tau + S(u) and tau = (e tau from the time channels) / e.
template <bool TIMED>
__device__ __forceinline__ TraceOut trace_ray(const TablesDev& T, float u, float delta,
                                             float alpha, float cotd, float u_ic, float u_oc) {
  TraceOut o;
  o.ncross = 0;
  o.ucr[0] = o.ucr[1] = 0.0f;
  o.tret[0] = o.tret[1] = 0.0f;
  o.mcr[0] = o.mcr[1] = 0;
  o.bits = 0;
  o.dprime = 0.0f;
  o.req = 0;
  float udot = -u * cotd;
  float e2 = udot * udot + u * u * (1.0f - u);
  float e = fsqrt(e2);
  o.e = e;
  if (e2 < kMu && u > 2.0f / 3.0f) {
    o.bits = BH_CAPTURED_BIT;
    return o;
  }
  int s = udot >= 0.0f ? 1 : -1;
  bool bound = e2 < kMu;
  float ua = bound ? apsis_f(e2) : 0.0f;
  float Dl = lookup_D(T, T.D, e2, u, ua, udot);
  o.req += 16;  // a bilinear fetch reads two pairs of adjacent floats
  float Da = 0.0f, phia = __builtin_inff();
  if (bound) {
    Da = lookup_D_apsis(T, T.D, e2);
    o.req += 8;
    phia = Da + 0.5f * kPi;
  }
  float ie = 0.0f, t_cam = 0.0f, t_a = 0.0f;
  if (TIMED) {
    ie = fdiv(1.0f, e);
    t_cam = lookup_D(T, T.Dt, e2, u, ua, udot) * ie + time_singular(u);
    if (bound) t_a = lookup_D_apsis(T, T.Dt, e2) * ie + time_singular(ua);
  }
  float phi = Dl + (s == 1 ? kPi - delta : delta) + (float)s * alpha;
  float m0 = floorf(phi * (1.0f / kPi));
  float phi0 = phi - kPi * m0;
  float u0 = lookup_U(T, T.U, e2, e, phi0);
  o.req += 16;
  int sg = (u0 > u) - (u0 < u);
  if (phi0 < phia && u_oc <= u0 && u0 <= u_ic && sg == s) {
    o.ucr[0] = u0;
    o.ncross = 1;
    o.bits |= BH_CROSS0_BIT;
    if (TIMED) {
      o.tret[0] = (float)s * (lookup_U(T, T.Ut, e2, e, phi0) * ie + time_singular(u0) - t_cam);
      o.mcr[0] = (int)m0;
    }
  }
  if (bound && s == 1) {
    phi = 2.0f * phia - phi;
    float m1 = floorf(phi * (1.0f / kPi));
    float phi1 = phi - kPi * m1;
    float u1 = lookup_U(T, T.U, e2, e, phi1);
    o.req += 16;
    if (phi1 < phia && u_oc <= u1 && u1 <= u_ic) {
      float t1 = 0.0f;
      if (TIMED)
        t1 = 2.0f * t_a - t_cam - (lookup_U(T, T.Ut, e2, e, phi1) * ie + time_singular(u1));
      // static indices only: a dynamically indexed array would be placed in LDS
      if (o.ncross == 0) {
        o.ucr[0] = u1;
        o.tret[0] = t1;
        o.mcr[0] = (int)m1;
      } else {
        o.ucr[1] = u1;
        o.tret[1] = t1;
        o.mcr[1] = (int)m1;
      }
      o.ncross += 1;
      o.bits |= BH_CROSS1_BIT;
    }
  }
  if (udot > 0.0f) {
    if (bound) {
      Dl = 2.0f * Da - Dl;
    } else {
      o.bits |= BH_CAPTURED_BIT;
      return o;
    }
  }
  o.dprime = delta + Dl;
  return o;
}

// ---- ray marching in place of TraceRay: the ablation of Section 5 (method M3, Table 1)
// Classic fourth-order Runge-Kutta on (u, w = du/dphi), w' = 3/2 u^2 - u (eq. rayequation),
// with the constant step h = 2 pi / N and at most N steps.  Inside a step u is the cubic
// Hermite interpolant of the two end states; in t = s / h, with the slopes scaled by h,
// p(t) = ((c3 t + c2) t + a) t + p0.  Its first root places the escape (Newton from the
// secant), its value at alpha + m pi a disc crossing.  h < pi (N >= 3): a step passes at
// most one disc-plane angle.  A beam still travelling after N steps is drawn as captured.
__device__ __forceinline__ float march_acc(float u) { return u * fmaf(1.5f, u, -1.0f); }

__device__ __forceinline__ TraceOut march_ray(float u, float alpha, float cotd, float u_ic,
                                              float u_oc, int nsteps, float h) {
  TraceOut o;
  o.ncross = 0;
  o.ucr[0] = o.ucr[1] = 0.0f;
  o.tret[0] = o.tret[1] = 0.0f;
  o.mcr[0] = o.mcr[1] = 0;
  o.bits = 0;
  o.dprime = 0.0f;
  o.req = 0;
  float w = -u * cotd;
  o.e = fsqrt(w * w + u * u * (1.0f - u));
  if (fabsf(cotd) >= 1e6f) {
    // within 1e-6 of the radius: the beam moves along r only (a step in phi cannot follow
    // it); outward it escapes undeflected at delta' = delta ~ 1 / cot(delta), inward it falls
    if (cotd > 0.0f)
      o.dprime = fdiv(1.0f, cotd);
    else
      o.bits = BH_CAPTURED_BIT;
    return o;
  }
  const bool inward = w > 0.0f;  // an apsis (largest u) can lie ahead
  const float hh = 0.5f * h, h6 = h * (1.0f / 6.0f), ih = fdiv(1.0f, h);
  float phid = alpha > 0.0f ? alpha : alpha + kPi;  // next disc-plane angle ahead
  for (int n = 0; n < nsteps; ++n) {
    const float a1 = march_acc(u);
    const float u2 = fmaf(hh, w, u), w2 = fmaf(hh, a1, w), a2 = march_acc(u2);
    const float u3 = fmaf(hh, w2, u), w3 = fmaf(hh, a2, w), a3 = march_acc(u3);
    const float u4 = fmaf(h, w3, u), w4 = fmaf(h, a3, w), a4 = march_acc(u4);
    const float un = fmaf(h6, fmaf(2.0f, w2 + w3, w + w4), u);
    const float wn = fmaf(h6, fmaf(2.0f, a2 + a3, a1 + a4), w);
    const float phi = (float)n * h;
    const bool esc = un < 0.0f;
    const float td = (phid - phi) * ih;
    if (esc || td <= 1.0f) {
      const float A = h * w, B = h * wn;
      const float c3 = 2.0f * (u - un) + A + B, c2 = 3.0f * (un - u) - 2.0f * A - B;
      float tend = 1.0f;
      if (esc) {
        float t = fdiv(u, u - un);
#pragma unroll
        for (int it = 0; it < 3; ++it) {
          float p = fmaf(fmaf(fmaf(c3, t, c2), t, A), t, u);
          float dp = fmaf(fmaf(3.0f * c3, t, 2.0f * c2), t, A);
          t = clampf(t - fdiv(p, dp), 0.0f, 1.0f);
        }
        tend = t;
      }
      if (td <= tend) {
        const float ud = fmaf(fmaf(fmaf(c3, td, c2), td, A), td, u);
        if (ud >= u_oc && ud <= u_ic) {
          const float slope = fmaf(fmaf(3.0f * c3, td, 2.0f * c2), td, A);
          o.bits |= inward && slope < 0.0f ? BH_CROSS1_BIT : BH_CROSS0_BIT;
          if (o.ncross == 0) o.ucr[0] = ud;
          else o.ucr[1] = ud;
          o.ncross = min(o.ncross + 1, 2);
        }
        phid += kPi;
      }
      if (esc) {
        o.dprime = fmaf(tend, h, phi);
        return o;
      }
    }
    u = un;
    w = wn;
    if (u >= 1.0f) {
      o.bits |= BH_CAPTURED_BIT;
      return o;
    }
  }
  o.bits |= BH_CAPTURED_BIT | BH_UNFINISHED_BIT;
  return o;
}

__device__ __forceinline__ float disc_temperature(const ViewDev& v, float u) {
  if (v.T_law == 1) {
    float f = u * u * u * (1.0f - fsqrt(3.0f * u));
    return f > 0.0f ? v.T0 * fsqrt(fsqrt(f * v.T_norm)) : 0.0f;
  }
  return v.T0 * __builtin_amdgcn_exp2f(-v.T_exp * __log2f(3.0f * u));
}

// Partner of this lane inside its quad (DPP quad permutation, all lanes active): MASK 1
// swaps lanes 0<->1, 2<->3 (row partner), MASK 2 swaps 0<->2, 1<->3 (column partner).
template <int MASK>
__device__ __forceinline__ float quad_partner(float x) {
  constexpr int ctrl = MASK == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, true));
}

// (value at the quad partner) - (value here): the forward difference along the row
// (MASK 1) or column (MASK 2) on lanes at the quad's low side and its negative on the
// others.  Every use below is invariant under flipping the sign of all row (or all
// column) differences of a lane: footprint extents and the tent weights take |.|, and
// the solid angles are norms of cross products; IEEE negation is exact, so the results
// equal those of the forward differences bit for bit.
template <int MASK>
__device__ __forceinline__ float quad_diff(float x) {
  return quad_partner<MASK>(x) - x;
}

// atan2 over the whole circle, from the half-plane version
__device__ __forceinline__ float fatan2_any(float y, float x) {
  float r = fatan2_pos(fabsf(y), x);
  return y < 0.0f ? -r : r;
}

// Density of the procedural disc particles (Appendix B) at the hit point (ht, hr, hphi):
// particle j's point a = (hphi - phi_j(ht)) mod 2 pi, phi_j(t) = omega_j t + phi0_j, has
// u_a = u1 + (u2 - u1) sin^2(c_j (a + phi_j(ht))); d^2 = (a/pi - 1)^2 + (hr - 1/u_a)^2 and
// the particle adds (1 - d^2)^2 inside d < 1.  Particle records (two float4 each):
// (u1, u2 - u1, c, omega), (phi0, r_peri - 1, r_apo + 1, 0), sorted by r_peri - 1; the
// radial bounds skip particles that cannot reach d < 1.
__device__ __forceinline__ float disc_density(const ViewDev& v, float ht, float hr, float hphi) {
  const float k2Pi = 2.0f * kPi;
  float rho = 0.0f;
  // particles are sorted by the inner end of their radial reach; no particle before
  // pstart[bin of hr] reaches out to hr.  The wave starts at the smallest such index over
  // its active lanes and stops at the first particle whose reach starts beyond the largest
  // hr of its active lanes (an LDS minimum and maximum in the wave's own slots: one wave's
  // LDS operations complete in order), so the loop and its exit are wave-uniform and the
  // records are scalar loads; each lane tests its own hr against the particle's reach.
  __shared__ int wave_start[16], wave_hmax[16];
  int j0 = 0;
  float hmax = 0.0f;
  if (v.nparts > 0) {
    int* slot = &wave_start[threadIdx.x >> 6];
    int* hslot = &wave_hmax[threadIdx.x >> 6];
    *slot = v.nparts;
    *hslot = 0;
    atomicMin(slot, v.pstart[(int)fminf(hr * v.pscale, (float)v.pbins)]);
    atomicMax(hslot, __float_as_int(hr));  // hr > 0: its bit patterns order as its values
    j0 = __builtin_amdgcn_readfirstlane(*(volatile int*)slot);
    hmax = __int_as_float(__builtin_amdgcn_readfirstlane(*(volatile int*)hslot));
  }
  for (int j = j0; j < v.nparts; ++j) {
    const float4 p0 = v.parts[2 * j], p1 = v.parts[2 * j + 1];
    if (hmax < p1.y) break;  // this and every later particle starts beyond every lane's hr
    if (hr >= p1.y && hr <= p1.z) {
      float ph = fmaf(p0.w, ht, p1.x);
      float a = hphi - ph;
      a -= k2Pi * floorf(a * (1.0f / k2Pi));
      // sin^2 x = (1 - cos 2x) / 2, with the hardware cosine (argument in turns: 2x / 2 pi)
      const float c2 = __builtin_amdgcn_cosf(p0.z * (a + ph) * (1.0f / kPi));
      float ua = fmaf(p0.y, fmaf(-0.5f, c2, 0.5f), p0.x);
      float dr = hr - fdiv(1.0f, ua);
      float da = a * (1.0f / kPi) - 1.0f;
      float d2 = da * da + dr * dr;
      if (d2 < 1.0f) rho += (1.0f - d2) * (1.0f - d2);
    }
  }
  return rho;
}

// ---- area sources (Section 3.3.2 "Emitted light": nebulae and galaxies in a cube map) ----
// The paper reads them with the texture unit's anisotropic filtering over the beam's
// footprint; this is that filter written out.  The footprint is the parallelogram of
// directions d' + w d_w d' + h d_h d', |w|, |h| <= 1/2 (the pixel's box); its two axes are
// measured in level-0 texels on the face of d' (face Jacobian, Euclidean length); an
// N_maj x N_min grid of probes sits at the cell centres of the parallelogram, spaced no
// closer than half a level-0 texel: with s = max(l_min / 2, 1/2), N_maj = clamp(ceil(l_maj /
// s), 1, 16) along the longer axis and N_min = clamp(ceil(l_min / s), 1, 2) across it (so
// N_maj = ceil(2 l_maj / l_min) by 2 once l_min >= 1); every probe reads level
// lambda = log2(max(l_maj / N_maj, l_min / N_min)) - 1 trilinearly; the result is the probes'
// mean of (I, I T), or of (R, G, B) on a band map.  Each probe takes the face of its own
// direction, so footprints cross cube edges; bilinear coordinates are clamped to the face's
// outermost texel centres.

// Cube face of a direction: axis k = argmax |p_k| (the lowest on ties), face 2k + (p_k < 0);
// (pk, pa, pb) = (p_k, p_{(k+1)%3}, p_{(k+2)%3})
struct FaceOf {
  int k, face;
  float pk, pa, pb, m;  // m = |p_k|
};

__device__ __forceinline__ FaceOf face_of(float p0, float p1, float p2) {
  const float a0 = fabsf(p0), a1 = fabsf(p1), a2 = fabsf(p2);
  FaceOf f;
  f.k = 0;
  f.m = a0;
  if (a1 > f.m) { f.k = 1; f.m = a1; }
  if (a2 > f.m) { f.k = 2; f.m = a2; }
  f.pk = f.k == 0 ? p0 : (f.k == 1 ? p1 : p2);
  f.pa = f.k == 0 ? p1 : (f.k == 1 ? p2 : p0);
  f.pb = f.k == 0 ? p2 : (f.k == 1 ? p0 : p1);
  f.face = 2 * f.k + (f.pk < 0.0f);
  return f;
}

// texel types of the two map formats: (I, I T), and (R, G, B, 0) for band maps
template <bool BANDS> struct AreaTexel { using type = float2; };
template <> struct AreaTexel<true> { using type = float4; };

__device__ __forceinline__ float2 lerp_texel(float f, float2 a, float2 b) {
  return make_float2(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y));
}
__device__ __forceinline__ float4 lerp_texel(float f, float4 a, float4 b) {
  return make_float4(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y), fmaf(f, b.z - a.z, a.z),
                     0.0f);
}

// every channel of level L, bilinear, at face coordinates (U, V) of `face`
template <bool BANDS>
__device__ __forceinline__ typename AreaTexel<BANDS>::type area_fetch(const AreaDev& M, int L,
                                                                      int face, float U,
                                                                      float V) {
  using Tx = typename AreaTexel<BANDS>::type;
  const int nL = M.n0 >> L;
  const uint32_t level0 = 8u * ((uint32_t)M.n0 * (uint32_t)M.n0 - (uint32_t)nL * (uint32_t)nL);
  const Tx* t = (const Tx*)M.tex + level0 + (uint32_t)face * (uint32_t)nL * (uint32_t)nL;
  if (nL == 1) return t[0];
  const float fn = (float)nL, top = fn - 1.0f;
  const float x = clampf(fmaf(0.5f * fn, U + 1.0f, -0.5f), 0.0f, top);
  const float y = clampf(fmaf(0.5f * fn, V + 1.0f, -0.5f), 0.0f, top);
  const int i0 = min((int)x, nL - 2), j0 = min((int)y, nL - 2);
  const float fx = x - (float)i0, fy = y - (float)j0;
  const Tx* r0 = t + (uint32_t)j0 * (uint32_t)nL + (uint32_t)i0;
  const Tx a = r0[0], b = r0[1], c = r0[nL], e = r0[nL + 1];
  return lerp_texel(fy, lerp_texel(fx, a, b), lerp_texel(fx, c, e));
}

// length, in level-0 texels, of the face-coordinate change along direction change (xk, xa,
// xb) (components in the face's axis order) at d' (im = 1 / |d'_k|, sg = sign of d'_k,
// (U, V) of d')
__device__ __forceinline__ float area_axis(float im, float sg, float U, float V, float xk,
                                           float xa, float xb, float half_n0) {
  const float dU = (xa - U * sg * xk) * im, dV = (xb - V * sg * xk) * im;
  return half_n0 * fsqrt(dU * dU + dV * dV);
}

// mean (I, I T) of the map over the footprint of d' with axes dw, dh, or mean (R, G, B)
// of a band map (BANDS, into A, B, C)
template <bool BANDS>
__device__ __forceinline__ void area_filter(const AreaDev& M, float d0, float d1, float d2,
                                            float w0, float w1, float w2, float h0, float h1,
                                            float h2, float& A, float& B, float& Cc) {
  using Tx = typename AreaTexel<BANDS>::type;
  const FaceOf c = face_of(d0, d1, d2);
  const int k = c.k;
  auto perm = [k](float x0, float x1, float x2, float& xk, float& xa, float& xb) {
    xk = k == 0 ? x0 : (k == 1 ? x1 : x2);
    xa = k == 0 ? x1 : (k == 1 ? x2 : x0);
    xb = k == 0 ? x2 : (k == 1 ? x0 : x1);
  };
  float wk, wa, wb, hk, ha, hb;
  perm(w0, w1, w2, wk, wa, wb);
  perm(h0, h1, h2, hk, ha, hb);
  const float im = fdiv(1.0f, c.m), sg = c.pk < 0.0f ? -1.0f : 1.0f;
  const float U = c.pa * im, V = c.pb * im, half_n0 = 0.5f * (float)M.n0;
  const float la = area_axis(im, sg, U, V, wk, wa, wb, half_n0);
  const float lb = area_axis(im, sg, U, V, hk, ha, hb, half_n0);
  const bool swap = lb > la;
  const float lmaj = swap ? lb : la, lmin = swap ? la : lb;
  // the axes in world order (probes whose face is looked up) and in the face's order
  const float j0 = swap ? h0 : w0, j1 = swap ? h1 : w1, j2 = swap ? h2 : w2;   // major
  const float n0_ = swap ? w0 : h0, n1 = swap ? w1 : h1, n2 = swap ? w2 : h2;  // minor
  const float jk = swap ? hk : wk, ja = swap ? ha : wa, jb = swap ? hb : wb;
  const float nk = swap ? wk : hk, na = swap ? wa : ha, nb = swap ? wb : hb;
  const float spc = fmaxf(0.5f * lmin, 0.5f), ispc = fdiv(1.0f, spc);
  const int nmaj = (int)clampf(ceilf(lmaj * ispc), 1.0f, 16.0f);
  const int nmin = lmin * ispc > 1.0f ? 2 : 1;
  const float fmaj = (float)nmaj, fmin = (float)nmin;
  const float sp = fmaxf(fdiv(lmaj, fmaj), fdiv(lmin, fmin));
  float lam = sp > 0.0f ? __log2f(sp) - 1.0f : 0.0f;
  lam = clampf(lam, 0.0f, (float)(M.levels - 1));
  const int L0 = (int)lam, L1 = min(L0 + 1, M.levels - 1);
  const float fr = lam - (float)L0;
  const bool two = fr > 0.0f && L1 != L0;  // the second level has weight
  // The directions on one face form a convex set of (w, h) (an intersection of half-planes),
  // so when the parallelogram's four corners lie on the face of d', every probe does too and
  // its face coordinates follow from the axes in the face's order without a face lookup.
  bool one_face = true;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float sa_ = (q & 1) ? 0.5f : -0.5f, sb_ = (q & 2) ? 0.5f : -0.5f;
    const FaceOf f = face_of(fmaf(sb_, n0_, fmaf(sa_, j0, d0)), fmaf(sb_, n1, fmaf(sa_, j1, d1)),
                             fmaf(sb_, n2, fmaf(sa_, j2, d2)));
    one_face = one_face && f.face == c.face;
  }
  float sa = 0.0f, sb = 0.0f, sc = 0.0f;
  const float inv = fdiv(1.0f, fmaj);
  for (int i = 0; i < nmaj; ++i) {
    const float ta = fmaf((float)i + 0.5f, inv, -0.5f);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (b >= nmin) break;
      const float tb = nmin == 1 ? 0.0f : (b == 0 ? -0.25f : 0.25f);
      int face;
      float pu, pv;
      if (one_face) {
        const float pk = fmaf(tb, nk, fmaf(ta, jk, c.pk));
        const float ip = fdiv(1.0f, fabsf(pk));
        pu = fmaf(tb, na, fmaf(ta, ja, c.pa)) * ip;
        pv = fmaf(tb, nb, fmaf(ta, jb, c.pb)) * ip;
        face = c.face;
      } else {
        const FaceOf f = face_of(fmaf(tb, n0_, fmaf(ta, j0, d0)), fmaf(tb, n1, fmaf(ta, j1, d1)),
                                 fmaf(tb, n2, fmaf(ta, j2, d2)));
        const float ip = fdiv(1.0f, f.m);
        pu = f.pa * ip;
        pv = f.pb * ip;
        face = f.face;
      }
      const Tx v0 = area_fetch<BANDS>(M, L0, face, pu, pv);
      Tx v = v0;
      if (two) v = lerp_texel(fr, v0, area_fetch<BANDS>(M, L1, face, pu, pv));
      sa += v.x;
      sb += v.y;
      if constexpr (BANDS) sc += v.z;
    }
  }
  const float in = inv * (nmin == 1 ? 1.0f : 0.5f);
  A = sa * in;
  B = sb * in;
  Cc = sc * in;
}

// C_b(r, g, D) from the colour-shift table (Section 3.4.2; cshift.hip): log2 values read
// trilinearly, linearly in r and g and, between the two D nodes around D, linearly in 1 / D;
// r, g and log2 D clamped to the node range
__device__ __forceinline__ float3 cshift_lookup(const float4* __restrict__ tab, float r, float g,
                                                float D) {
  constexpr float top = (float)(kCshiftN - 1), step = 6.0f / (float)(kCshiftN - 1);
  const float x = clampf(r * top, 0.0f, top), y = clampf(g * top, 0.0f, top);
  const int i0 = min((int)x, kCshiftN - 2), j0 = min((int)y, kCshiftN - 2);
  const float fx = x - (float)i0, fy = y - (float)j0;
  const float Dc = clampf(D, 0.125f, 8.0f);
  const int k0 = min((int)((__log2f(Dc) + 3.0f) * (1.0f / step)), kCshiftN - 2);
  const float inv0 = exp2f(3.0f - (float)k0 * step), inv1 = exp2f(3.0f - (float)(k0 + 1) * step);
  const float fz = clampf(fdiv(fdiv(1.0f, Dc) - inv0, inv1 - inv0), 0.0f, 1.0f);
  const float4* p = tab + ((uint32_t)i0 * kCshiftN + (uint32_t)j0) * kCshiftN + (uint32_t)k0;
  constexpr uint32_t si = kCshiftN * kCshiftN, sj = kCshiftN;
  const float4 c000 = p[0], c001 = p[1], c010 = p[sj], c011 = p[sj + 1];
  const float4 c100 = p[si], c101 = p[si + 1], c110 = p[si + sj], c111 = p[si + sj + 1];
  const float4 e = lerp_texel(fx, lerp_texel(fy, lerp_texel(fz, c000, c001),
                                             lerp_texel(fz, c010, c011)),
                              lerp_texel(fy, lerp_texel(fz, c100, c101),
                                         lerp_texel(fz, c110, c111)));
  return make_float3(exp2f(e.x), exp2f(e.y), exp2f(e.z));
}

// One pixel; every lane of the wave must call this together (quad exchanges).
// COUNT: also mark every star-map texel the footprint visits and add up the bytes the pixel
// requests (measurement only, see CountBufs).  ANIM: views may have a particle disc
// (retarded times).
// MARCH: ray marching (march_ray) in place of TraceRay; no tables are read.
template <bool COUNT, bool ANIM = false, bool MARCH = false, int AREA = 0>
__device__ __forceinline__ void render_pixel(const ViewDev& v, const TablesDev& T,
                                             const LutDev& L, int px, int py,
                                             const CountBufs* cnt) {

  // ---- beam initialisation (Section 3.2)
  float qw = (float)px + 0.5f - v.half_w;
  float qh = v.half_h - (float)py - 0.5f;
  float inq = __builtin_amdgcn_rsqf(qw * qw + qh * qh + v.f * v.f);  // argument >= f^2 > 0
  float q0 = qw * inq, q1 = qh * inq, q2 = -v.f * inq;
  // camera direction and its aberration into the static frame, as the part transverse to
  // e_x' (n0, n1, n2) and the radial component nr
  float nc0 = q0 * v.ew[0] + q1 * v.eh[0] + q2 * v.ed[0];
  float nc1 = q0 * v.ew[1] + q1 * v.eh[1] + q2 * v.ed[1];
  float nc2 = q0 * v.ew[2] + q1 * v.eh[2] + q2 * v.ed[2];
  float ncr = q0 * v.er[0] + q1 * v.er[1] + q2 * v.er[2];
  float nv = nc0 * v.vhat[0] + nc1 * v.vhat[1] + nc2 * v.vhat[2] + ncr * v.er[3];
  float ka = (v.gamma - 1.0f) * nv - v.gamma * v.vmag;
  // coordinate direction d: the transverse part as is, the radial component scaled by
  // sqrt(1 - u) (eq. staticbasis)
  const float d0 = nc0 + ka * v.vhat[0], d1 = nc1 + ka * v.vhat[1], d2 = nc2 + ka * v.vhat[2];
  const float dr = v.sq1mu * (ncr + ka * v.er[3]);
  float dcam = fdiv(v.inv_sq1mu, v.gamma * (1.0f - v.vmag * nv));
  // e_z' = e_x' x d / |e_x' x d|, and |e_x' x d| = |transverse part|
  float cz0 = v.rhat[1] * d2 - v.rhat[2] * d1;
  float cz1 = v.rhat[2] * d0 - v.rhat[0] * d2;
  float cz2 = v.rhat[0] * d1 - v.rhat[1] * d0;
  const float ncz2 = d0 * d0 + d1 * d1 + d2 * d2;
  const float dn2 = ncz2 + dr * dr;
  float ncz, inv_ncz;  // |e_x' x d| and its inverse
  float ey0, ey1, ey2;  // e_y' = e_z' x e_x'
  unsigned bits = 0;
  float u_ic = v.u_ic, u_oc = v.u_oc;
  if (!(ncz2 > 1e-14f * dn2)) {
    // radial beam: any plane through it; pick one containing a fixed axis
    bits |= BH_DEGENERATE_BIT;
    float ax0 = fabsf(v.rhat[0]) < 0.9f ? 1.0f : 0.0f, ax1 = 1.0f - ax0;
    cz0 = v.rhat[1] * 0.0f - v.rhat[2] * ax1;
    cz1 = v.rhat[2] * ax0 - v.rhat[0] * 0.0f;
    cz2 = v.rhat[0] * ax1 - v.rhat[1] * ax0;
    float n2 = __builtin_amdgcn_rsqf(cz0 * cz0 + cz1 * cz1 + cz2 * cz2);
    cz0 *= n2; cz1 *= n2; cz2 *= n2;
    ey0 = cz1 * v.rhat[2] - cz2 * v.rhat[1];
    ey1 = cz2 * v.rhat[0] - cz0 * v.rhat[2];
    ey2 = cz0 * v.rhat[1] - cz1 * v.rhat[0];
    ncz = fmaxf(fsqrt(ncz2), 1e-7f * fsqrt(dn2));
    inv_ncz = fdiv(1.0f, ncz);
    u_ic = -1.0f;
  } else {
    inv_ncz = __builtin_amdgcn_rsqf(ncz2);
    ncz = ncz2 * inv_ncz;
    cz0 *= inv_ncz; cz1 *= inv_ncz; cz2 *= inv_ncz;
    // (e_x' x d) x e_x' is d's transverse part
    ey0 = d0 * inv_ncz; ey1 = d1 * inv_ncz; ey2 = d2 * inv_ncz;
  }
  float delta = fatan2_pos(ncz, dr);
  // t = +-(e_z x e_z') with t.e_y' >= 0; alpha = angle(e_x', t)
  float t0 = -cz1, t1 = cz0;
  float nt = fsqrt(t0 * t0 + t1 * t1);
  float alpha = 0.0f;
  if (!(nt > 1e-7f)) {
    bits |= BH_DEGENERATE_BIT;
    u_ic = -1.0f;
  } else {
    float int_ = fdiv(1.0f, nt);
    float tx = (t0 * v.rhat[0] + t1 * v.rhat[1]) * int_;
    float ty = (t0 * ey0 + t1 * ey1) * int_;
    if (ty < 0.0f) {
      tx = -tx;
      ty = -ty;
      t0 = -t0;  // t now points along the line of nodes with t.e_y' >= 0
      t1 = -t1;
    }
    alpha = fatan2_pos(ty, tx);
  }
  float zeta = cz2;

  // ---- TraceRay (Algorithm 1)
  const float cotd = dr * inv_ncz;
  TraceOut tr;
  if constexpr (MARCH)
    tr = march_ray(v.u_c, alpha, cotd, u_ic, u_oc, v.march_steps, v.march_h);
  else
    tr = trace_ray<ANIM>(T, v.u_c, delta, alpha, cotd, u_ic, u_oc);
  bits |= tr.bits;
  const bool captured = (tr.bits & BH_CAPTURED_BIT) != 0;
  uint32_t req = tr.req;  // bytes requested (COUNT only)

  // ---- disc (Sections 3.3.3, 3.4.2), front to back
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, trans = 1.0f;
  if (tr.ncross > 0) {
    const float ie = fdiv(1.0f, tr.e);
    // animated disc: crossing k sits at (-1)^m_k t, i.e. at disc azimuth az0 + m_k pi
    const bool anim = ANIM && v.density_mode == 1;
    float az0 = 0.0f;
    if (anim) az0 = fatan2_any(t1, t0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      // a crossing behind an opaque one (transmittance exactly 0) adds nothing
      if (k >= tr.ncross || !(trans > 0.0f)) break;
      float uk = k == 0 ? tr.ucr[0] : tr.ucr[1];
      float Tp = disc_temperature(v, uk);
      // 1 / k'^t = sqrt(1 - 3u/2) and Omega' = sqrt(u^3 / 2) on the circular orbit at u
      float ikt = fsqrt(1.0f - 1.5f * uk);
      float om = fsqrt(0.5f * uk * uk * uk);
      float D = dcam * ikt * fdiv(1.0f, 1.0f + om * zeta * ie);
      float4 Lb = band_lookup(L, D * Tp);
      if (COUNT) req += 32;  // two band-table entries
      float rk = v.rho;
      if (anim) {
        float tk = k == 0 ? tr.tret[0] : tr.tret[1];
        int mk = k == 0 ? tr.mcr[0] : tr.mcr[1];
        float dens = disc_density(v, v.time - tk, fdiv(1.0f, uk), az0 + (float)mk * kPi);
        rk = fminf(1.0f, v.rho * dens);
      }
      float w = trans * rk * v.k_disc;
      cr += w * Lb.x;
      cg += w * Lb.y;
      cb += w * Lb.z;
      trans *= 1.0f - rk;
    }
  }

  // ---- stars (Sections 3.3.2, 3.4.1)
  // hardware sine and cosine (argument in turns): the escape direction only places star
  // light, where their ~1e-6 rad error is a thousandth of a pixel
  const float turns = tr.dprime * 0.159154943091895336f;
  const float sdp = __builtin_amdgcn_sinf(turns), cdp = __builtin_amdgcn_cosf(turns);
  float dp0 = captured ? 0.0f : cdp * v.rhat[0] + sdp * ey0;
  float dp1 = captured ? 0.0f : cdp * v.rhat[1] + sdp * ey1;
  float dp2 = captured ? 0.0f : cdp * v.rhat[2] + sdp * ey2;
  int cap = captured ? 1 : 0;
  cap |= __builtin_amdgcn_mov_dpp(cap, 0xB1, 0xF, 0xF, true);
  cap |= __builtin_amdgcn_mov_dpp(cap, 0x4E, 0xF, 0xF, true);
  float dw0 = quad_diff<1>(dp0), dw1 = quad_diff<1>(dp1), dw2 = quad_diff<1>(dp2);
  float dh0 = quad_diff<2>(dp0), dh1 = quad_diff<2>(dp1), dh2 = quad_diff<2>(dp2);
  int mip = 255;
  if (cap) bits |= BH_STAR_ZEROED_BIT;
  if (v.has_stars && !cap) {
    const StarsDev& S = v.stars;
    float a0 = fabsf(dp0), a1 = fabsf(dp1), a2 = fabsf(dp2);
    int k = 0;
    float m = a0;
    if (a1 > m) { k = 1; m = a1; }
    if (a2 > m) { k = 2; m = a2; }
    float dk = k == 0 ? dp0 : (k == 1 ? dp1 : dp2);
    float da = k == 0 ? dp1 : (k == 1 ? dp2 : dp0);
    float db = k == 0 ? dp2 : (k == 1 ? dp0 : dp1);
    float wk = k == 0 ? dw0 : (k == 1 ? dw1 : dw2);
    float wa = k == 0 ? dw1 : (k == 1 ? dw2 : dw0);
    float wb = k == 0 ? dw2 : (k == 1 ? dw0 : dw1);
    float hk = k == 0 ? dh0 : (k == 1 ? dh1 : dh2);
    float ha = k == 0 ? dh1 : (k == 1 ? dh2 : dh0);
    float hb = k == 0 ? dh2 : (k == 1 ? dh0 : dh1);
    int face = 2 * k + (dk < 0.0f);
    float sgk = dk < 0.0f ? -1.0f : 1.0f;
    float im = fdiv(1.0f, m);
    float U = da * im, V = db * im;
    float J00 = (wa - U * sgk * wk) * im, J01 = (ha - U * sgk * hk) * im;
    float J10 = (wb - V * sgk * wk) * im, J11 = (hb - V * sgk * hk) * im;
    float hu = fabsf(J00) + fabsf(J01), hv = fabsf(J10) + fabsf(J11);
    float E0 = fmaxf(hu, hv) * (float)S.n0;
    // smallest level with E0 / 2^L <= 8: from the exponent and mantissa of E0 / 8
    int Lv = 0;
    {
      float q = E0 * 0.125f;
      if (q > 1.0f) {
        unsigned b = __float_as_uint(q);
        int ex = (int)((b >> 23) & 255u) - 127;   // q = 1.m * 2^ex, q finite and > 1
        Lv = ex + ((b & 0x7fffffu) != 0u ? 1 : 0);
      }
      if (!(q <= 3.0e38f)) Lv = S.levels - 1;      // infinite or NaN footprint
      Lv = min(Lv, S.levels - 1);
    }
    mip = Lv;
    float det = J00 * J11 - J01 * J10;
    // band-colour star maps are read only by the band variants (AREA 2 and 3)
    const bool bands = AREA >= 2 && S.bands;
    float A = 0.0f, B = 0.0f, Cb = 0.0f;
    // behind an opaque disc crossing (transmittance exactly 0) the stars add nothing: their
    // light is scaled by trans below, so the gather is skipped (the level above is kept)
    if (fabsf(det) >= 1e-20f && trans > 0.0f) {
      float idet = fdiv(1.0f, det);
      Footprint F;
      // inverse face Jacobian
      const float i00 = J11 * idet, i01 = -J01 * idet, i10 = -J10 * idet, i11 = J00 * idet;
      const int nL = S.n0 >> Lv;
      const float fn = (float)nL;
      // clamp before the integer conversion (equal to floor-then-clamp for in-range values)
      const float top = fn - 1.0f;
      int x0 = (int)clampf(0.5f * (U - hu + 1.0f) * fn, 0.0f, top);
      int x1 = (int)clampf(0.5f * (U + hu + 1.0f) * fn, 0.0f, top);
      int y0 = (int)clampf(0.5f * (V - hv + 1.0f) * fn, 0.0f, top);
      int y1 = (int)clampf(0.5f * (V + hv + 1.0f) * fn, 0.0f, top);
      x1 = min(x1, x0 + 8);
      y1 = min(y1, y0 + 8);
      F.nL = nL;
      const int wpr = ((nL + 31) >> 5) + 1;
      F.wpr4 = 4 * wpr;
      F.sh = x0 & 31;
      F.ny = y1 - y0;
      F.span = (1u << (x1 - x0 + 1)) - 1u;  // x1 - x0 <= 8
      F.texel0 = S.level_off[Lv] + ((uint32_t)face * (uint32_t)nL + (uint32_t)y0) * (uint32_t)nL +
                 (uint32_t)x0;
      F.occ = S.occ + S.occ_off[Lv] +
              2u * (((uint32_t)face * (uint32_t)nL + (uint32_t)y0) * (uint32_t)wpr +
                    (uint32_t)(x0 >> 5));
      // a level-L texel is tw = 2 / nL wide in face coordinates; the corner (x0, y0) lies at
      // (cu, cv) from the centre direction (U, V)
      const float tw = __builtin_ldexpf(S.tw0, Lv);  // nL = n0 / 2^L: 2 / nL exactly
      const float cu = (float)x0 * tw - 1.0f - U, cv = (float)y0 * tw - 1.0f - V;
      F.Wc = i00 * tw;
      F.Wr = i01 * tw;
      F.W0 = fmaf(i00, cu, i01 * cv);
      F.Hc = i10 * tw;
      F.Hr = i11 * tw;
      F.H0 = fmaf(i10, cu, i11 * cv);
      F.one = S.one;
      if (COUNT) req += 12;  // level offsets and scale
      if constexpr (AREA >= 2) {
        if (bands) {
          if (S.fp16)
            gather<kTexBand16, COUNT>(S.tex, F, cnt, req, A, B, Cb);
          else
            gather<kTexBand32, COUNT>(S.tex, F, cnt, req, A, B, Cb);
        }
      }
      if (!bands) {
        if (S.fp16)
          gather<kTexIT16, COUNT, AREA != 3>(S.tex, F, cnt, req, A, B, Cb);
        else
          gather<kTexIT32, COUNT, AREA != 3>(S.tex, F, cnt, req, A, B, Cb);
      }
      const float iscale = S.scale[Lv];
      A *= iscale;
      B *= S.fp16 && !bands ? iscale * 1024.0f : iscale;
      Cb *= iscale;
    }
    float cdx = dw1 * dh2 - dw2 * dh1, cdy = dw2 * dh0 - dw0 * dh2, cdz = dw0 * dh1 - dw1 * dh0;
    // Omega / Omega' = |q_w x q_h| / |d'_w x d'_h| with the same quad differences of the
    // camera-frame direction q = (q^w, q^h, -f) inq.  The row partner shares q^h and the
    // column partner q^w, so with a = quad difference of inq along the row and b along the
    // column, q_w = (dq0, q^h a, -f a) and q_h = (q^w b, dq1, -f b), whose cross product is
    // (f a (dq1 - q^h b), f b (dq0 - q^w a), dq0 dq1 - q^w q^h a b).
    const float qa = quad_diff<1>(inq), qb = quad_diff<2>(inq);
    const float dq0 = quad_diff<1>(q0), dq1 = quad_diff<2>(q1);
    const float cq0 = v.f * qa * (dq1 - qh * qb), cq1 = v.f * qb * (dq0 - qw * qa);
    const float cq2 = dq0 * dq1 - (qw * qh) * (qa * qb);
    const float om2 = cq0 * cq0 + cq1 * cq1 + cq2 * cq2;
    const float omp2 = cdx * cdx + cdy * cdy + cdz * cdz;
    if (bands) {
      // light of any colour: band sum and chromaticity, shifted by C(r, g, D_cam)
      const float Ssum = A + B + Cb;
      if (Ssum > 0.0f && omp2 > 0.0f) {
        const float iS = fdiv(1.0f, Ssum);
        const float3 C = cshift_lookup(S.ctab, A * iS, B * iS, dcam);
        const float sc = trans * v.k_star * fsqrt(om2) * __builtin_amdgcn_rsqf(omp2) * Ssum;
        cr += sc * C.x;
        cg += sc * C.y;
        cb += sc * C.z;
      }
    } else if (A > 0.0f && omp2 > 0.0f) {
      float Tpix = fdiv(B, A);
      float4 Lr = band_lookup(L, dcam * Tpix);
      float4 Ln = band_lookup(L, Tpix);
      if (COUNT) req += 64;
      float sc = trans * v.k_star * fsqrt(om2) * __builtin_amdgcn_rsqf(omp2) * fdiv(A, Ln.w);
      cr += sc * Lr.x;
      cg += sc * Lr.y;
      cb += sc * Lr.z;
    }
  }

  // ---- area sources: the footprint's mean radiance, one Doppler shift per pixel as for
  // stars, no lensing amplification (Section 3.4.1)
  if ((AREA == 1 || AREA == 2) && v.area.tex && !cap && trans > 0.0f) {
    float A, B, Cc;
    if (AREA == 2 && v.area.bands) {
      // light of any colour: band sum S and chromaticity (r, g), shifted by C(r, g, D_cam)
      area_filter<true>(v.area, dp0, dp1, dp2, dw0, dw1, dw2, dh0, dh1, dh2, A, B, Cc);
      const float S = A + B + Cc;
      if (S > 0.0f) {
        const float iS = fdiv(1.0f, S);
        const float3 C = cshift_lookup(v.area.ctab, A * iS, B * iS, dcam);
        const float sc = trans * v.area.k_area * S;
        cr += sc * C.x;
        cg += sc * C.y;
        cb += sc * C.z;
      }
    } else {
      area_filter<false>(v.area, dp0, dp1, dp2, dw0, dw1, dw2, dh0, dh1, dh2, A, B, Cc);
      if (A > 0.0f) {
        const float Tpix = fdiv(B, A);
        const float4 Lr = band_lookup(L, dcam * Tpix), Ln = band_lookup(L, Tpix);
        const float sc = trans * v.area.k_area * fdiv(A, Ln.w);
        cr += sc * Lr.x;
        cg += sc * Lr.y;
        cb += sc * Lr.z;
      }
    }
  }

  if (COUNT) {
    if (px < v.width && py < v.height) req += v.aov ? 32 : 16;
    unsigned long long t = req;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(cnt->l2_bytes, t);
  }
  if (px < v.width && py < v.height) {
    size_t idx = (size_t)py * v.width + px;
    store_stream(&v.out[idx], make_float4(cr, cg, cb, 1.0f));
    if (v.aov) {
      bits |= (unsigned)mip << 8;
      store_stream(&v.aov[idx], make_float4(captured ? __builtin_inff() : tr.dprime, tr.ucr[0],
                                             tr.ucr[1], __uint_as_float(bits)));
    }
  }
}

template <int TW, int TH, int PPT>
struct TileCfg {
  static constexpr int kBX = TW / 8, kBY = TH / 8;           // 8x8 blocks per tile
  static constexpr int kWaves = kBX * kBY / PPT;
  static constexpr int kThreads = 64 * kWaves;
  static_assert(kBX * kBY % PPT == 0, "blocks must divide by pixels per thread");
  static_assert(kWaves <= 16, "the particle loop keeps one LDS slot per wave, 16 at most");
};

template <int TW, int TH, int PPT, bool COUNT = false, bool ANIM = false, bool MARCH = false,
          int AREA = 0>
__device__ __forceinline__ void render_tile(const ViewDev& v, const TablesDev& T, const LutDev& L,
                                            int tx0, int ty0, const CountBufs* cnt = nullptr) {
  using C = TileCfg<TW, TH, PPT>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane >> 2;
  const int ox = 2 * (q & 3) + (lane & 1), oy = 2 * (q >> 2) + ((lane >> 1) & 1);
#pragma unroll 1
  for (int p = 0; p < PPT; ++p) {
    int blk = p * C::kWaves + wave;
    int bx = blk % C::kBX, by = blk / C::kBX;
    int px = tx0 + 8 * bx + ox, py = ty0 + 8 * by + oy;
    // skip 8x8 blocks entirely outside the image (uniform per wave)
    if (tx0 + 8 * bx >= v.width || ty0 + 8 * by >= v.height) continue;
    render_pixel<COUNT, ANIM, MARCH, AREA>(v, T, L, px, py, cnt);
  }
}

// XCD-aware tile order.  Workgroup b runs on XCD b % 8.  The image's tiles are grouped in
// blocks of kXBW x kXBH tiles that stay on one XCD (neighbouring tiles share that XCD's L2),
// and the blocks are dealt to the 8 XCDs in turn, so every XCD gets work from all over the
// image: per-tile cost varies strongly across a frame (shadow, disc, star field), and one
// band of rows per XCD left the lightest XCDs idle for ~10% of the frame.
constexpr int kXBW = 4, kXBH = 2;

__device__ __forceinline__ bool xcd_tile(int b, int tiles_x, int tiles_y, int* col, int* row) {
  int x = b & 7, k = b >> 3;
  int bx = (tiles_x + kXBW - 1) / kXBW;
  int blk = x + 8 * (k / (kXBW * kXBH)), q = k % (kXBW * kXBH);
  *row = (blk / bx) * kXBH + q / kXBW;
  *col = (blk % bx) * kXBW + q % kXBW;
  return *col < tiles_x && *row < tiles_y;
}

// workgroups of a plain launch over tiles_x x tiles_y tiles (a multiple of 8)
static inline int xcd_grid(int tiles_x, int tiles_y) {
  int nblk = ((tiles_x + kXBW - 1) / kXBW) * ((tiles_y + kXBH - 1) / kXBH);
  return ((nblk + 7) / 8) * 8 * kXBW * kXBH;
}

// Resident waves per SIMD the one-launch and per-tile kernels are held to (the register
// budget the compiler keeps to): 8, and 6 for the area-source variants, whose probe loop
// spilled 20 vector registers to memory at 8 waves and ran 17% faster at 6 without spills,
// 5 when they also read band colours.  Band star maps without area maps fit 8 (64 VGPRs).
template <int FEAT>
constexpr int kMinWaves = (FEAT & kFeatArea) ? ((FEAT & kFeatBands) ? 5 : 6) : 8;

// the area and band code a feature set needs (render_pixel's AREA): 0 none, 1 (I, I T) area
// maps, 2 area maps of either format and band star maps (run-time branches on the maps'
// formats), 3 band star maps without area maps
template <int FEAT>
constexpr int kAreaOf =
    (FEAT & kFeatBands) ? ((FEAT & kFeatArea) ? 2 : 3) : ((FEAT & kFeatArea) ? 1 : 0);

// One launch per view, tiles in the XCD-aware order above.
// At least 8 resident waves per SIMD: the register budget the compiler keeps to.  The
// animated variant would otherwise take 92 scalar registers and fit only 7 waves; held to
// 8 it spills a few scalars into vector-register lanes and runs 7% faster.  (The
// persistent batch kernel is left unbounded: held to 8 waves it would spill to memory.)
template <int TW, int TH, int PPT, int FEAT>
__global__ void __launch_bounds__((TW / 8) * (TH / 8) * 64 / PPT, kMinWaves<FEAT>)
    k_render(ViewDev v, TablesDev T, LutDev L, int tiles_x, int tiles_y) {
  int col, row;
  if (!xcd_tile(blockIdx.x, tiles_x, tiles_y, &col, &row)) return;
  render_tile<TW, TH, PPT, false, (FEAT & kFeatParticles) != 0, false, kAreaOf<FEAT>>(
      v, T, L, col * TW, row * TH);
}

// The render with ray marching in place of TraceRay (16x16 tiles, one pixel per thread);
// AREA as in render_pixel.
template <int AREA>
__global__ void __launch_bounds__(256)
    k_render_march(ViewDev v, LutDev L, int tiles_x, int tiles_y) {
  int col, row;
  if (!xcd_tile(blockIdx.x, tiles_x, tiles_y, &col, &row)) return;
  TablesDev none{};
  render_tile<16, 16, 1, false, false, true, AREA>(v, none, L, col * 16, row * 16);
}

// The run holding flat tile index `it` (wave-uniform): the last run whose start is <= it.
__device__ __forceinline__ TileRun find_run(const TileRun* __restrict__ runs, int nruns,
                                            int it) {
  int lo = 0, hi = nruns - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane(runs[mid].start) <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  TileRun r = runs[lo];
  r.view = __builtin_amdgcn_readfirstlane(r.view);
  r.tile0 = __builtin_amdgcn_readfirstlane(r.tile0);
  r.start = __builtin_amdgcn_readfirstlane(r.start);
  r.tiles_x = __builtin_amdgcn_readfirstlane(r.tiles_x);
  return r;
}

template <int TW, int TH, int PPT, int FEAT>
__device__ __forceinline__ void render_flat_tile(const ViewDev* __restrict__ views,
                                                 const TileRun* __restrict__ runs, int nruns,
                                                 int it, const TablesDev& T, const LutDev& L) {
  TileRun r = find_run(runs, nruns, it);
  int tile = r.tile0 + (it - r.start);
  // fields are read through the reference as they are needed (wave-uniform scalar loads):
  // a copy of the whole record would hold ~65 scalar registers across the tile
  const ViewDev& v = views[r.view];
  render_tile<TW, TH, PPT, false, (FEAT & kFeatParticles) != 0, false, kAreaOf<FEAT>>(
      v, T, L, (tile % r.tiles_x) * TW,
                                        (tile / r.tiles_x) * TH);
}

// Persistent launch over the tiles of many views.  Every wave works on its own: it claims
// indices from an atomic counter and renders every 8x8 block of the tiles a claim covers,
// so no claim waits on a barrier and the workgroup shape (4 waves) is the same for every
// tile configuration.  Claim j < nbig covers claim_tiles consecutive flat tiles (about 16
// blocks); the last `tail` tiles (4 per wave) go one per claim, so the launch does not end
// waiting on a few long claims.  A wave leaves at its first claim past the last tile; the
// counter only grows, so every wave reaches that exit.  Held to 7 resident waves per SIMD:
// the loop over tiles keeps ~14 more vector registers live than one tile does, so at 8
// waves it would spill; the host sizes the grid to 7 waves per SIMD.
constexpr int kBatchThreads = 256;

template <int TW, int TH, int PPT, int FEAT>
__global__ void __launch_bounds__(kBatchThreads, 7)
    k_render_batch(const ViewDev* __restrict__ views, const TileRun* __restrict__ runs,
                   int nruns, int ntiles, int* __restrict__ counter, TablesDev T, LutDev L) {
  using C = TileCfg<TW, TH, 1>;
  constexpr int kBlocks = C::kBX * C::kBY;                // 8x8 blocks per tile
  constexpr int claim_tiles = kBlocks >= 16 ? 1 : 16 / kBlocks;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 2;
  const int ox = 2 * (q & 3) + (lane & 1), oy = 2 * (q >> 2) + ((lane >> 1) & 1);
  const int tail = min(ntiles, 4 * (int)(gridDim.x * (kBatchThreads / 64)));
  const int nbig = (ntiles - tail) / claim_tiles;          // tiles [0, claim_tiles nbig)
  const int first_single = claim_tiles * nbig;
  for (;;) {
    int j = 0;
    if (lane == 0) j = atomicAdd(counter, 1);
    j = __builtin_amdgcn_readfirstlane(j);                 // lane 0's claim, the wave's
    int it0, it1;
    if (j < nbig) {
      it0 = claim_tiles * j;
      it1 = it0 + claim_tiles;
    } else {
      it0 = first_single + (j - nbig);
      it1 = it0 + 1;
    }
    if (it0 >= ntiles) break;
#pragma unroll 1
    for (int it = it0; it < it1; ++it) {
      const TileRun r = find_run(runs, nruns, it);
      const int tile = r.tile0 + (it - r.start);
      const ViewDev& v = views[r.view];
      const int tx0 = (tile % r.tiles_x) * TW, ty0 = (tile / r.tiles_x) * TH;
#pragma unroll 1
      for (int blk = 0; blk < kBlocks; ++blk) {
        const int bx = tx0 + 8 * (blk % C::kBX), by = ty0 + 8 * (blk / C::kBX);
        if (bx >= v.width || by >= v.height) continue;    // block outside the image
        render_pixel<false, (FEAT & kFeatParticles) != 0, false, kAreaOf<FEAT>>(
            v, T, L, bx + ox, by + oy, nullptr);
      }
    }
  }
}

// Tiles of many views without persistence: one workgroup per flat tile index.  Chunks of
// kXChunk consecutive flat tiles (a row segment of one view) stay on one XCD and the chunks
// are dealt to the 8 XCDs in turn, as in the plain launch.
constexpr int kXChunk = kXBW * kXBH;

template <int TW, int TH, int PPT, int FEAT>
__global__ void __launch_bounds__((TW / 8) * (TH / 8) * 64 / PPT, kMinWaves<FEAT>)
    k_render_list(const ViewDev* __restrict__ views, const TileRun* __restrict__ runs,
                  int nruns, int ntiles, TablesDev T, LutDev L) {
  int b = blockIdx.x;
  int k = b >> 3;
  int it = (k / kXChunk) * (8 * kXChunk) + (b & 7) * kXChunk + k % kXChunk;
  if (it >= ntiles) return;
  render_flat_tile<TW, TH, PPT, FEAT>(views, runs, nruns, it, T, L);
}

__global__ void k_reset_counter(int* c) { *c = 0; }

// Measurement variant of the plain launch (16x16 tiles): marks the star-map texels that
// the footprints visit.
__global__ void __launch_bounds__(256)
    k_render_count(ViewDev v, TablesDev T, LutDev L, int tiles_x, int ntiles, CountBufs cnt) {
  int tile = blockIdx.x;
  if (tile >= ntiles) return;
  render_tile<16, 16, 1, true>(v, T, L, (tile % tiles_x) * 16, (tile / tiles_x) * 16, &cnt);
}

__global__ void k_popcount(const uint32_t* __restrict__ bits, int64_t n,
                           unsigned long long* __restrict__ total) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned c = i < n ? __popc(bits[i]) : 0u;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(total, (unsigned long long)c);
}

// TraceRay alone, for unit tests: rays = [u, delta, alpha, u_ic, u_oc].  TIMED also writes
// (retarded time 0, retarded time 1, m_0, m_1) per ray to out_time.
template <bool TIMED>
__global__ void k_trace_rays(TablesDev T, const float* __restrict__ rays, int64_t n,
                             float4* __restrict__ out, float4* __restrict__ out_time) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* r = rays + 5 * i;
  float u = r[0], delta = r[1];
  float sd, cd;
  sincosf(delta, &sd, &cd);
  TraceOut t = trace_ray<TIMED>(T, u, delta, r[2], cd / sd, r[3], r[4]);
  bool cap = (t.bits & BH_CAPTURED_BIT) != 0;
  out[i] = make_float4(cap ? __builtin_inff() : t.dprime, t.ucr[0], t.ucr[1],
                       __uint_as_float(t.bits));
  if (TIMED)
    out_time[i] = make_float4(t.tret[0], t.tret[1], (float)t.mcr[0], (float)t.mcr[1]);
}

__global__ void __launch_bounds__(256)
    k_march_rays(const float* __restrict__ rays, int64_t n, int nsteps, float h,
                 float4* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* r = rays + 5 * i;
  float sd, cd;
  sincosf(r[1], &sd, &cd);
  // a radial beam (delta = 0 or pi) keeps a finite slope, as in the render path
  TraceOut t = march_ray(r[0], r[2], cd / fmaxf(sd, 1e-7f), r[3], r[4], nsteps, h);
  bool cap = (t.bits & BH_CAPTURED_BIT) != 0;
  out[i] = make_float4(cap ? __builtin_inff() : t.dprime, t.ucr[0], t.ucr[1],
                       __uint_as_float(t.bits));
}

// ---- scratch of the allocation-free batched launch -------------------------------------------
// Device memory of bh_render_batch_noalloc: the persistent form's claim counter (first 256
// bytes), then up to kNoAllocViews view records and as many tile runs.  A file-scope device
// array: each GPU the library runs on holds its own copy until the process ends, and every
// call on that GPU shares it (it keeps the last call's contents; the counter is reset by a
// kernel before each persistent launch).  In host code `scratch` only names the symbol: its
// device address comes from scratch_address(), once per device.
constexpr int kNoAllocViews = BH_NOALLOC_MAX_VIEWS;
constexpr size_t kNoAllocHead = 256;
constexpr size_t kNoAllocBytes =
    kNoAllocHead + (size_t)kNoAllocViews * (sizeof(ViewDev) + sizeof(TileRun));
static_assert(sizeof(ViewDev) % 16 == 0, "view records keep the tile runs 16-byte aligned");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Address of `scratch` on the current device (call with that device current).
hipError_t scratch_address(void** p) {
  return hipGetSymbolAddress(p, HIP_SYMBOL(scratch));
}

// ---- host-side launchers ------------------------------------------------------------------

struct TileEntry {
  int tw, th, waves, ppt;
  // indexed by the features the views may use: kFeatParticles | kFeatArea | kFeatBands
  // (kFeatBands alone: band star maps without area maps)
  void (*plain[8])(const ViewDev&, const TablesDev&, const LutDev&, hipStream_t);
  void (*batch[8])(const ViewDev*, const TileRun*, int, int, int*, const TablesDev&,
                   const LutDev&, int grid, hipStream_t);
  void (*list[8])(const ViewDev*, const TileRun*, int, int, const TablesDev&, const LutDev&,
                  hipStream_t);
};

template <int TW, int TH, int PPT, int FEAT>
static void launch_plain(const ViewDev& v, const TablesDev& T, const LutDev& L, hipStream_t s) {
  using C = TileCfg<TW, TH, PPT>;
  int tiles_x = (v.width + TW - 1) / TW, tiles_y = (v.height + TH - 1) / TH;
  hipLaunchKernelGGL((k_render<TW, TH, PPT, FEAT>), dim3(xcd_grid(tiles_x, tiles_y)),
                     dim3(C::kThreads), 0, s, v, T, L, tiles_x, tiles_y);
}

template <int TW, int TH, int PPT, int FEAT>
static void launch_batch(const ViewDev* views, const TileRun* runs, int nruns, int ntiles,
                         int* counter, const TablesDev& T, const LutDev& L, int grid,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
  hipLaunchKernelGGL((k_render_batch<TW, TH, PPT, FEAT>), dim3(grid), dim3(kBatchThreads), 0, s,
                     views, runs, nruns, ntiles, counter, T, L);
}

template <int TW, int TH, int PPT, int FEAT>
static void launch_list(const ViewDev* views, const TileRun* runs, int nruns, int ntiles,
                        const TablesDev& T, const LutDev& L, hipStream_t s) {
  using C = TileCfg<TW, TH, PPT>;
  int grid = (ntiles + 8 * kXChunk - 1) / (8 * kXChunk) * (8 * kXChunk);
  hipLaunchKernelGGL((k_render_list<TW, TH, PPT, FEAT>), dim3(grid), dim3(C::kThreads), 0, s,
                     views, runs, nruns, ntiles, T, L);
}

#define BH_FEATS(F, TW, TH, PPT)                                                          \
  {F<TW, TH, PPT, 0>, F<TW, TH, PPT, 1>, F<TW, TH, PPT, 2>, F<TW, TH, PPT, 3>,             \
   F<TW, TH, PPT, 4>, F<TW, TH, PPT, 5>, F<TW, TH, PPT, 6>, F<TW, TH, PPT, 7>}
#define BH_TILE(TW, TH, PPT)                                                                \
  {TW, TH, TileCfg<TW, TH, PPT>::kWaves, PPT, BH_FEATS(launch_plain, TW, TH, PPT),          \
   BH_FEATS(launch_batch, TW, TH, PPT), BH_FEATS(launch_list, TW, TH, PPT)}

static const TileEntry kTiles[] = {
    BH_TILE(16, 16, 1), BH_TILE(32, 8, 1), BH_TILE(16, 8, 1), BH_TILE(8, 8, 1),
    BH_TILE(32, 16, 2), BH_TILE(16, 16, 2), BH_TILE(32, 32, 4), BH_TILE(64, 16, 4),
};

int tile_config_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
void tile_config(int i, int* tw, int* th, int* waves, int* ppt) {
  *tw = kTiles[i].tw;
  *th = kTiles[i].th;
  *waves = kTiles[i].waves;
  *ppt = kTiles[i].ppt;
}

hipError_t launch_render(int cfg, const ViewDev& v, const TablesDev& T, const LutDev& L,
                         hipStream_t s) {
  kTiles[cfg].plain[view_features(v)](v, T, L, s);
  return hipGetLastError();
}

// persistent != 0: `grid` persistent workgroups pulling tiles from an atomic counter;
// otherwise one workgroup per tile.
hipError_t launch_render_batch(int cfg, int persistent, int feat, const ViewDev* views,
                               const TileRun* runs, int nruns, int ntiles, int* counter,
                               const TablesDev& T, const LutDev& L, int grid, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int a = feat & (kFeatParticles | kFeatArea | kFeatBands);
  if (persistent)
    kTiles[cfg].batch[a](views, runs, nruns, ntiles, counter, T, L, grid, s);
  else
    kTiles[cfg].list[a](views, runs, nruns, ntiles, T, L, s);
  return hipGetLastError();
}

hipError_t launch_render_count(const ViewDev& v, const TablesDev& T, const LutDev& L,
                               uint32_t* touched, int64_t words, unsigned long long* total,
                               unsigned long long* l2_bytes, hipStream_t s) {
  int tiles_x = (v.width + 15) / 16, ntiles = tiles_x * ((v.height + 15) / 16);
  hipLaunchKernelGGL(k_render_count, dim3(ntiles), dim3(256), 0, s, v, T, L, tiles_x, ntiles,
                     CountBufs{touched, l2_bytes});
  hipLaunchKernelGGL(k_popcount, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, touched,
                     words, total);
  return hipGetLastError();
}

hipError_t launch_render_march(const ViewDev& v, const LutDev& L, hipStream_t s) {
  int tiles_x = (v.width + 15) / 16, tiles_y = (v.height + 15) / 16;
  const dim3 grid(xcd_grid(tiles_x, tiles_y));
  if ((v.area.tex && v.area.bands) || (v.has_stars && v.stars.bands))
    hipLaunchKernelGGL(k_render_march<2>, grid, dim3(256), 0, s, v, L, tiles_x, tiles_y);
  else if (v.area.tex)
    hipLaunchKernelGGL(k_render_march<1>, grid, dim3(256), 0, s, v, L, tiles_x, tiles_y);
  else
    hipLaunchKernelGGL(k_render_march<0>, grid, dim3(256), 0, s, v, L, tiles_x, tiles_y);
  return hipGetLastError();
}

hipError_t launch_march_rays(const float* rays, int64_t n, int nsteps, float h, float4* out,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_march_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rays, n,
                     nsteps, h, out);
  return hipGetLastError();
}

hipError_t launch_trace_rays(const TablesDev& T, const float* rays, int64_t n, float4* out,
                             float4* out_time, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256));
  if (out_time)
    hipLaunchKernelGGL(k_trace_rays<true>, grid, dim3(256), 0, s, T, rays, n, out, out_time);
  else
    hipLaunchKernelGGL(k_trace_rays<false>, grid, dim3(256), 0, s, T, rays, n, out, out_time);
  return hipGetLastError();
}

}  // namespace bh
