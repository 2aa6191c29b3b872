// vc_device.hpp -- inline single-precision codec for the MI355X kernels.
//
// Encodes a float32 3-vector into one 64-bit word and back, following
// Trojak & Witherden (arXiv 2003.02633):
//   spherical coordinates                    §2.1, Eqs. (cart2sphere, spherical)
//   angle quantisation, round half up        §2.1, Eq. (a_disc) and the nint definition
//   reconstruction                           §2.1, Eq. (a_inv)
//   shortened exponent/mantissa magnitude    §2.3
//   bit layouts <s,e,m>-p-t                  §2.3, Fig. (comp_regimes)
//   fractional split                         §2.4, Eq. (q_split)
//   tanh / cosine companding                 §2.5
//
// Two encoders with the same contract (every level exact except within one single-precision ulp
// of the angle from a level boundary; the magnitude rounded to nearest-even from the exact norm):
//   * FP64-assisted (the default, encode_vec64): squares, norm and ratios in FP64 (on gfx950
//     an FP64 FMA issues like an FP32 one), an rsqrt / reciprocal seed with one correction
//     step, an octant reduction to |b| <= tan(pi/8) and a degree-4 polynomial for
//     atan(b)/b - 1 (relative error 2.5e-9), the level coordinate and its floor in FP64.
//     Norms within 2^-44 of a rounding midpoint take an exact 128-bit integer path.
//   * single precision (encode_vec32, FP32 + integer only): the same steps with double-float
//     (pairs of FP32) arithmetic; the level coordinate is exact to ~2^-24 level units, and
//     norms within 2^-14 grid units of a midpoint (about 3 in 10^5) take the exact path.
// In both, the half-up ties of the axis directions (theta = 0, phi = pi/2) come out exactly.
// A layout with the truncating magnitude (L0722T) instead rounds the norm to nearest-even at
// 24 bits, the float32 magnitude, and drops its trailing 23 - m mantissa bits (§2.3 as printed).
// Decode: hardware sin/cos in revolutions (v_sin_f32 / v_cos_f32) of an exactly formed level
// offset, accuracy ~3e-7 of |x|; the dot product of two codes is taken in spherical form.
//
// The header also compiles for the host (VC_HOST_EMULATION) with libm stand-ins
// for the AMDGPU builtins, so the integer and control logic can be exercised
// on a CPU.
#pragma once

#include <stdint.h>

#ifdef VC_HOST_EMULATION
#include <math.h>
#include <string.h>
#define VC_DI inline
#define VC_NOINL
#else
#include <hip/hip_runtime.h>
#define VC_DI __device__ __forceinline__
#define VC_NOINL __device__ __noinline__
#endif

#include "vc_coeffs.inc"

namespace vc {

// ------------------------------------------------------------------ primitives
#ifdef VC_HOST_EMULATION
VC_DI uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
VC_DI float ubits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
VC_DI float rsq_(float x) { return (float)(1.0 / sqrt((double)x)); }
VC_DI float rcp_(float x) { return (float)(1.0 / (double)x); }
VC_DI float sin_rev(float r) { return (float)sin(6.283185307179586 * (double)r); }
VC_DI float cos_rev(float r) { return (float)cos(6.283185307179586 * (double)r); }
VC_DI int frexp_exp(float x) { int e; frexpf(x, &e); return e; }
VC_DI float ldexp_(float x, int e) { return ldexpf(x, e); }
VC_DI float floor_(float x) { return floorf(x); }
VC_DI float fma_(float a, float b, float c) { return fmaf(a, b, c); }
VC_DI float log2_(float x) { return log2f(x); }
VC_DI float sqrt_(float x) { return sqrtf(x); }
#else
VC_DI uint32_t fbits(float f) { return __float_as_uint(f); }
VC_DI float ubits(uint32_t u) { return __uint_as_float(u); }
VC_DI float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
VC_DI float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
VC_DI float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }   // sin(2 pi r)
VC_DI float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }   // cos(2 pi r)
VC_DI int frexp_exp(float x) { return __builtin_amdgcn_frexp_expf(x); }
VC_DI float ldexp_(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
VC_DI float floor_(float x) { return __builtin_floorf(x); }
VC_DI float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
VC_DI float log2_(float x) { return __builtin_amdgcn_logf(x); }     // v_log_f32 (log2)
VC_DI float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }   // v_sqrt_f32
#endif
#ifdef VC_HOST_EMULATION
VC_DI uint64_t dbits(double d) { uint64_t u; memcpy(&u, &d, 8); return u; }
VC_DI double dfrom_bits(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }
VC_DI double rsq64_(double x) { return (1.0 / sqrt(x)) * (1.0 + 3e-8); }   // crude, like v_rsq_f64
VC_DI double rcp64_(double x) { return (1.0 / x) * (1.0 - 4e-8); }
VC_DI double floor64_(double x) { return floor(x); }
VC_DI double fma64_(double a, double b, double c) { return fma(a, b, c); }
#else
VC_DI uint64_t dbits(double d) { return (uint64_t)__double_as_longlong(d); }
VC_DI double dfrom_bits(uint64_t u) { return __longlong_as_double((long long)u); }
VC_DI double rsq64_(double x) { return __builtin_amdgcn_rsq(x); }   // v_rsq_f64, ~2^-24
VC_DI double rcp64_(double x) { return __builtin_amdgcn_rcp(x); }   // v_rcp_f64, ~2^-24
VC_DI double floor64_(double x) { return __builtin_floor(x); }
VC_DI double fma64_(double a, double b, double c) { return __builtin_fma(a, b, c); }
#endif
// max / min of two doubles that are never signalling NaNs: the plain v_max_f64 / v_min_f64,
// without the operand canonicalisation the compiler adds for fmax / fmin in IEEE mode.  A quiet
// NaN in the first operand gives the second (as the hardware's IEEE minNum/maxNum does).
#ifdef VC_HOST_EMULATION
VC_DI double fmax64_nn(double a, double b) { return a > b ? a : b; }
VC_DI double fmin64_nn(double a, double b) { return a < b ? a : b; }
#else
VC_DI double fmax64_nn(double a, double b) { double r; asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b)); return r; }
VC_DI double fmin64_nn(double a, double b) { double r; asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b)); return r; }
#endif
// A level coordinate about to be converted to an integer, from an encoder path whose result is
// discarded for non-finite input (the slow path of the caller replaces it).  On the GPU the
// conversion of a NaN or an infinity is a defined instruction (0 or saturation) and the value is
// never used; the host build, where such a conversion is undefined, clamps it first.
#ifdef VC_HOST_EMULATION
VC_DI double level_guard(double q) { return fmin64_nn(q, 0x1p30); }
#else
VC_DI double level_guard(double q) { return q; }
#endif
VC_DI float fabs_(float x) { return ubits(fbits(x) & 0x7fffffffu); }
#ifdef VC_HOST_EMULATION
VC_DI float fmax_(float a, float b) { return fmaxf(a, b); }
VC_DI float fmin_(float a, float b) { return fminf(a, b); }
// NaN-propagating maximum / minimum (IEEE 754-2019), unlike fmax / fmin, which drop a NaN
VC_DI float fmaximum_(float a, float b) { return (a != a || b != b) ? NAN : fmaxf(a, b); }
VC_DI float fminimum_(float a, float b) { return (a != a || b != b) ? NAN : fminf(a, b); }
#else
VC_DI float fmax_(float a, float b) { return __builtin_fmaxf(a, b); }
VC_DI float fmin_(float a, float b) { return __builtin_fminf(a, b); }
// NaN-propagating maximum / minimum (IEEE 754-2019; v_maximum3_f32 / v_minimum3_f32 on gfx950),
// unlike fmax / fmin, which drop a NaN
VC_DI float fmaximum_(float a, float b) { return __builtin_elementwise_maximum(a, b); }
VC_DI float fminimum_(float a, float b) { return __builtin_elementwise_minimum(a, b); }
#endif
// the WIDTH bits of x from bit OFF on, as one v_bfe_u32 (the compiler splits a constant-field
// extract into a shift and a mask)
template <int OFF, int WIDTH>
VC_DI uint32_t ubfe_(uint32_t x)
{
  static_assert(OFF >= 0 && WIDTH > 0 && OFF + WIDTH <= 32, "field within 32 bits");
#ifdef VC_HOST_EMULATION
  return (x >> OFF) & (WIDTH == 32 ? ~0u : (1u << WIDTH) - 1u);
#else
  uint32_t r;
  asm("v_bfe_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(OFF), "i"(WIDTH));
  return r;
#endif
}
VC_DI uint32_t umax3(uint32_t a, uint32_t b, uint32_t c) { uint32_t m = a > b ? a : b; return m > c ? m : c; }

// ------------------------------------------------------------------ layouts
// <S,E,M>-P-T with exponent bias BIAS; fields MSB->LSB: sign, exponent,
// mantissa, n_phi, n_theta (Fig. comp_regimes).  TR selects the magnitude rounding of the
// encoder: 0 nearest-even from the exact norm at 1+M bits, 1 the float32 magnitude (nearest-even
// at 24 bits) with its trailing 23 - M bits dropped.  Decoding does not depend on it.
template <int S_, int E_, int M_, int P_, int T_, int BIAS_, int TR_ = 0>
struct Layout {
  static constexpr int s = S_, e = E_, m = M_, p = P_, t = T_, bias = BIAS_;
  static constexpr bool trunc = TR_ != 0;
  static constexpr int mr = trunc ? 23 : M_;          // fraction bits the norm is rounded to
  static constexpr int sh_p = T_, sh_m = T_ + P_, sh_e = T_ + P_ + M_;
  static constexpr uint32_t emask = (1u << E_) - 1u;
  static constexpr int emax = (int)emask - 1;         // all-ones exponent is reserved
  static constexpr bool keep_sub = (E_ == 8 && BIAS_ == 127);
  static constexpr uint64_t reserved = (uint64_t)emask << sh_e;
  // largest finite magnitude: E = emax, M all ones (E and M fields only)
  static constexpr uint64_t saturated = ((uint64_t)(emask - 1u) << sh_e) | (((1ull << M_) - 1ull) << sh_m);
  static_assert(S_ + E_ + M_ + P_ + T_ == 64, "layout must fill 64 bits");
  static_assert(M_ == 22 || M_ == 23, "mantissa of 22 or 23 bits");
  static_assert(!TR_ || (M_ < 23 && !keep_sub), "truncation drops bits only below 23; no subnormal codes");
};
using L0722 = Layout<0, 7, 22, 17, 18, 80>;
using L0722T = Layout<0, 7, 22, 17, 18, 80, 1>;     // <0,7,22>-17-18, truncating magnitude
using L0723 = Layout<0, 7, 23, 17, 17, 80>;
using L0823 = Layout<0, 8, 23, 16, 17, 127>;
using L1823 = Layout<1, 8, 23, 16, 16, 127>;

enum Mode { PLAIN = 0, TANH = 1, COS = 2, FRAC = 3 };

// Per-codec constants, filled on the host (vc_api.cpp) and passed by value.
struct Params {
  uint32_t nmax_t, nmax_p;   // n_theta_max, n_phi_max
  uint32_t T;                // fractional split: n_theta_max + 1 (0 otherwise)
  uint32_t base_t;           // theta: (n_max+1)/2 if odd, n_max/2 if even
  uint32_t odd_t;            // 1 if n_theta_max is odd
  uint32_t comp_t, comp_p;   // companding applied to theta / phi
  uint32_t pad0;
  uint64_t limit;            // fractional split: P*T (codes >= limit are invalid)
  // encode, level units: theta |Q| = Kt |theta|/pi, phi V = Np phi/pi + 1/2
  float Kt;                  // n_theta_max / 2
  float Np;                  // n_phi_max
  float Ct_h, Ct_l;          // (n_theta_max/2)/pi as a double-float
  float Cp_h, Cp_l;          // n_phi_max/pi as a double-float
  // decode, revolutions
  float rt_h, rt_l;          // 1/n_theta_max as a double-float
  float rp_h, rp_l;          // 1/(2 n_phi_max) as a double-float
  float half_t;              // n_theta_max / 2
  // companding
  float gam, inv_gam, cgam;  // gamma, 1/gamma, tanh(gamma)
  float w[8];                // tanh: h(u)/u - 1 = sum w[i] (u^2)^i (u in [-1,1])
  int wdeg;
  // FP64-assisted encode
  int wdeg64;
  double Kt64, Np64;         // n_theta_max/2, n_phi_max
  double Ct64, Cp64;         // (n_theta_max/2)/pi, n_phi_max/pi
  double invKt64, invKc64;   // 1/(n_theta_max/2), 1/(n_phi_max/2)
  double invT64;             // fractional split: RN64(1/T) (decode quotient)
  double w64[16];            // tanh: h(u)/u = sum w64[i] (u^2)^i
  // companding with the single-precision encoder: the level boundaries of the companded
  // coordinate in the uniform one, T[j] = K h^-1(j / K) as double-float pairs (T[2j], T[2j+1]),
  // j = 0 .. floor(K) + 1 (T[0] = 0, the last +huge); theta (K = n_theta_max / 2) and phi
  // (K = n_phi_max / 2).  Device (or, in the host build, host) memory owned by the library.
  const float* ctab_t;
  const float* ctab_p;
};

enum Prec { PREC_F32 = 0, PREC_F64 = 1 };

// ------------------------------------------------------------------ decode

// Magnitude r_hat = (1 + M/2^m) 2^(E - b) of a code, an exact float32 bit pattern (§2.3); zero for
// E = 0 (IEEE subnormals for the layouts that keep them), NaN for the reserved all-ones exponent.
// The E and M fields are adjacent in the high word (E above M), so one shift and mask place them
// as the float's exponent and leading mantissa bits.
template <class L>
VC_DI float decode_mag(uint64_t w)
{
  static_assert(L::sh_m >= 32, "E and M fields in the high word");
  const uint32_t hi = (uint32_t)(w >> 32);
  const uint32_t em = ubfe_<L::sh_m - 32, L::e + L::m>(hi);
  const uint32_t rbits = L::keep_sub ? em << (23 - L::m)                       // the IEEE value itself
                                     : (em << (23 - L::m)) + ((uint32_t)(127 - L::bias) << 23);
  float r = ubits(rbits);
  const uint32_t Eb = hi & (L::emask << (L::sh_e - 32));                   // E in place
  if (!L::keep_sub && Eb == 0u) r = 0.0f;
  if (Eb == (L::emask << (L::sh_e - 32))) r = ubits(0x7fc00000u);          // reserved -> NaN
  return r;
}

// The magnitude bits alone, for codes that are neither the zero code nor the reserved code
// (special_code false): decode_mag without its two selects.
template <class L>
VC_DI float decode_mag_fast(uint64_t w)
{
  const uint32_t hi = (uint32_t)(w >> 32);
  const uint32_t em = ubfe_<L::sh_m - 32, L::e + L::m>(hi);
  return ubits(L::keep_sub ? em << (23 - L::m) : (em << (23 - L::m)) + ((uint32_t)(127 - L::bias) << 23));
}

// The codes whose magnitude is not (1 + M/2^m) 2^(E - b): the zero code (E = 0, for layouts
// without subnormal codes) and the reserved code (E all ones).
template <class L>
VC_DI bool special_code(uint64_t w)
{
  constexpr int es = L::sh_e - 32;
  const uint32_t hi = (uint32_t)(w >> 32);
  if constexpr (L::keep_sub) {
    return (hi & (L::emask << es)) == (L::emask << es);
  } else {
    // E is the top field of the word (no sign bit): E - 1 wraps below 1 and reaches emask - 1
    // at the reserved exponent, whatever the mantissa bits below it
    static_assert(L::s == 0, "layouts without subnormal codes have no sign bit");
    return hi - (1u << es) >= ((L::emask - 1u) << es);
  }
}

// The fields of a code: magnitude r_hat (NaN for codes past the fractional split's limit) and
// the level counts n_theta, n_phi (Eq. q_split for the fractional split).
template <class L, int MODE, bool FAST = false>
VC_DI void decode_fields(uint64_t w, const Params& P, float& r, uint32_t& nth, uint32_t& nph)
{
  r = FAST ? decode_mag_fast<L>(w) : decode_mag<L>(w);
  if (MODE == FRAC) {
    const uint64_t np = w & ((1ull << (L::p + L::t)) - 1ull);
    if (np >= P.limit) r = ubits(0x7fc00000u);
    // n_phi = floor(np / T), n_theta = np mod T.  np < 2^35 is exact in a double (its bits placed
    // in the mantissa of 2^52); with invT64 = RN64(1/T) the product is within 2^-27 of np / T
    // (np / T < 2^24), while np / T lies at least 1/T >= 2^-24 from the next integer above, so
    // the truncated estimate is the quotient or, when T divides np, one less: one upward
    // correction of the 32-bit remainder (< 2 T <= 2^25) finishes it.  The clamp keeps the
    // conversion in range for codes past the limit (their magnitude is NaN).
    const double npd = dfrom_bits(0x4330000000000000ull | np) - 0x1p52;
    const uint32_t q0 = (uint32_t)fmin64_nn(npd * P.invT64, 0x1p25);
    const uint32_t rem = (uint32_t)np - q0 * P.T;
    const bool up = rem >= P.T;
    nph = up ? q0 + 1u : q0;
    nth = up ? rem - P.T : rem;
  } else {
    nth = (uint32_t)w & ((1u << L::t) - 1u);
    nph = (uint32_t)(w >> L::sh_p) & ((1u << L::p) - 1u);
  }
}

// Magnitude of a code as a norm sees it: r_hat (decode_mag), and NaN for fractional-split codes
// past the limit P T, which decode to NaN (Eq. q_split has no level pair for them).
template <class L, int MODE>
VC_DI float decode_mag_checked(uint64_t w, const Params& P)
{
  float r = decode_mag<L>(w);
  if (MODE == FRAC && (w & ((1ull << (L::p + L::t)) - 1ull)) >= P.limit) r = ubits(0x7fc00000u);
  return r;
}

// A level count times 1/n_max (or 1/(2 n_max)).  For the uniform levels of every layout
// n_max = 2^k - 1 (k = 16..18), so 1/n_max = 2^-k (1 + 2^-k + 2^-2k + ...) and its float32
// rounding 2^-k (1 + 2^-k) is off by 2^-2k <= 2^-32 relative: one product is rounded as well as
// the exact one.  The fractional split's n_max = T - 1 is arbitrary and takes the double-float
// reciprocal (h + l).
template <int MODE>
VC_DI float times_rcp(float x, float h, float l)
{
  if (MODE == FRAC) return fma_(x, h, x * l);
  return x * h;
}

// Angles of the levels in revolutions (Eq. a_inv; §2.5 for the tanh map):
// theta_hat/(2 pi) = n/n_max - 1/2, phi_hat/(2 pi) = n/(2 n_max) for uniform levels.  (The
// cosine map has no call here: its sines and cosines are algebraic in the levels, cos_map_trig.)
template <int MODE>
VC_DI void level_revs(uint32_t nth, uint32_t nph, const Params& P, float& rev_t, float& rev_p)
{
  static_assert(MODE != COS, "the cosine map decodes through cos_map_trig");
  // theta: (n - n_max/2)/n_max = n/n_max - 1/2, one FMA with the single-product reciprocal;
  // the fractional split forms n - n_max/2 exactly and takes the double-float reciprocal
  auto theta_rev = [&]() {
    if (MODE == FRAC) return times_rcp<MODE>((float)nth - P.half_t, P.rt_h, P.rt_l);
    return fma_((float)nth, P.rt_h, -0.5f);
  };
  if (MODE == TANH) {
    // the centred level coordinate h = 2 n/n_max - 1 maps back to u = atanh(c h)/gamma
    // (c = tanh gamma), taken as (log2(1 + c h) - log2(1 - c h)) ln 2/(2 gamma): two hardware
    // logarithms, no division; theta_hat = pi u, phi_hat = pi (u + 1)/2
    auto inv = [&](uint32_t n, float two_over_nmax) {
      const float a = P.cgam * fma_((float)n, two_over_nmax, -1.0f);
      return (log2_(1.0f + a) - log2_(1.0f - a)) * (0.34657359f * P.inv_gam);
    };
    if (P.comp_t) rev_t = 0.5f * inv(nth, 2.0f * P.rt_h);
    else rev_t = theta_rev();
    if (P.comp_p) rev_p = fma_(0.25f, inv(nph, 4.0f * P.rp_h), 0.25f);
    else rev_p = times_rcp<MODE>((float)nph, P.rp_h, P.rp_l);
  } else {
    rev_t = theta_rev();
    rev_p = times_rcp<MODE>((float)nph, P.rp_h, P.rp_l);
  }
}

// Sines and cosines of the decoded angles under the cosine map (§2.5): with the centred level
// coordinates h = 2 n_t/N_t - 1 and g = 2 n_p/N_p - 1 (N the level counts), theta_hat = 2 asin(h)
// and phi_hat = pi/2 + asin(g), so
//   cos theta = 1 - 2 h^2,  sin theta = 2 h sqrt(1 - h^2),  cos phi = -g,  sin phi = sqrt(1 - g^2),
// where 1 - h^2 = 4 n (N - n)/N^2 comes from the exact factors n and N - n (no cancellation at
// the ends, and sin phi = 0 exactly at the poles).  An angle outside the companding mask takes
// the uniform levels and the hardware sine and cosine.
VC_DI void cos_map_trig(uint32_t nth, uint32_t nph, const Params& P, float& st, float& ct, float& sp, float& cp)
{
  if (P.comp_t) {
    const float n = (float)nth, m = (float)(P.nmax_t - nth);
    const float h = fma_(n, 2.0f * P.rt_h, -1.0f);
    ct = fma_(-2.0f * h, h, 1.0f);
    st = (4.0f * P.rt_h) * h * sqrt_(n * m);
  } else {
    const float rev = fma_((float)nth, P.rt_h, -0.5f);
    st = sin_rev(rev);
    ct = cos_rev(rev);
  }
  if (P.comp_p) {
    const float n = (float)nph, m = (float)(P.nmax_p - nph);
    cp = fma_(n, -4.0f * P.rp_h, 1.0f);
    sp = (4.0f * P.rp_h) * sqrt_(n * m);
  } else {
    const float rev = (float)nph * P.rp_h;
    sp = sin_rev(rev);
    cp = cos_rev(rev);
  }
}

// Cartesian vector of a code: Eq. (a_inv) then Eq. (cart2sphere).
// FAST: for codes with special_code false only (the magnitude without the zero and reserved
// cases)
template <class L, int MODE, bool FAST = false>
VC_DI void decode_vec(uint64_t w, const Params& P, float& ox, float& oy, float& oz)
{
  float r;
  uint32_t nth, nph;
  decode_fields<L, MODE, FAST>(w, P, r, nth, nph);
  float st, ct, sp, cp;
  if constexpr (MODE == COS) {
    cos_map_trig(nth, nph, P, st, ct, sp, cp);
  } else {
    float rev_t, rev_p;
    level_revs<MODE>(nth, nph, P, rev_t, rev_p);
    st = sin_rev(rev_t);
    ct = cos_rev(rev_t);
    sp = sin_rev(rev_p);
    cp = cos_rev(rev_p);
  }
  const float rs = r * sp;
  ox = rs * ct;
  oy = rs * st;
  oz = r * cp;
}

// decode(a) . decode(b) in spherical form (Eq. cart2sphere):
//   r_a r_b (sin phi_a sin phi_b cos(theta_a - theta_b) + cos phi_a cos phi_b),
// five hardware sine/cosine evaluations instead of the eight of two decodes.  For uniform theta
// levels the difference of the angles is formed from the exact difference of the level counts.
// The cosine map, whose decode needs no sine or cosine, takes the Cartesian product.
template <class L, int MODE>
VC_DI float dot_pair(uint64_t wa, uint64_t wb, const Params& P)
{
  if constexpr (MODE == COS) {
    float ax, ay, az, bx, by, bz;
    decode_vec<L, MODE>(wa, P, ax, ay, az);
    decode_vec<L, MODE>(wb, P, bx, by, bz);
    return fma_(ax, bx, fma_(ay, by, az * bz));
  } else {
    float ra, rb;
    uint32_t ta, pa, tb, pb;
    decode_fields<L, MODE>(wa, P, ra, ta, pa);
    decode_fields<L, MODE>(wb, P, rb, tb, pb);
    float rta, rpa, rtb, rpb, drev;
    level_revs<MODE>(ta, pa, P, rta, rpa);
    level_revs<MODE>(tb, pb, P, rtb, rpb);
    if (MODE == PLAIN || MODE == FRAC || (MODE == TANH && !P.comp_t))
      drev = times_rcp<MODE>((float)((int)ta - (int)tb), P.rt_h, P.rt_l);   // |ta - tb| < 2^24: exact
    else
      drev = rta - rtb;
    const float sa = sin_rev(rpa), ca = cos_rev(rpa), sb = sin_rev(rpb), cb = cos_rev(rpb);
    return (ra * rb) * fma_(sa * sb, cos_rev(drev), ca * cb);
  }
}

// The companding mask (which angles the map applies to) is a run-time field.  A kernel runs its
// body as with_compand_mask<MODE>(P, body): when both angles are companded (the default) the body
// gets a copy of the parameters whose mask is a compile-time constant, so its per-vector code has
// no branches on it; other masks take the run-time tests.
template <int MODE, class F>
VC_DI void with_compand_mask(const Params& P, F&& body)
{
  if constexpr (MODE == TANH || MODE == COS) {
    if (P.comp_t && P.comp_p) {
      Params Q = P;
      Q.comp_t = 1u;
      Q.comp_p = 1u;
      body(static_cast<const Params&>(Q));
    } else {
      body(P);
    }
  } else {
    body(P);
  }
}

// Degree of the tanh map's polynomial an encoder instantiation evaluates (TDEG of encode_vec): the
// host fits the smallest degree it needs (8 up to gamma ~0.55, at most 15; higher coefficients
// zero) and launches the instantiation of this bound that covers it.
inline constexpr int tanh_tdeg(int fitted) { return fitted <= 8 ? 8 : 15; }

// ------------------------------------------------------------------ encode helpers

// Exact round-to-nearest-even of sqrt(x^2+y^2+z^2) to `prec` significant bits
// (grid never finer than 2^-149 when keep_sub), by integer arithmetic on the
// float bit patterns.  Returns the integer significand j and grid exponent g
// with r_hat = j 2^g (j == 0 for the zero vector).
struct NormRound {
  uint32_t j;   // significand (j == 0 for the zero vector)
  int g;        // grid exponent: r_hat = j 2^g; NORM_NONFINITE for non-finite input
};
constexpr int NORM_NONFINITE = -0x7fffffff;
// (returned by value, in registers: the call of this rare path needs no stack frame)
VC_NOINL NormRound exact_norm_round(float x, float y, float z, int prec, bool keep_sub)
{
  uint32_t Mf[3], Ef[3];
  const float c[3] = {x, y, z};
  if (umax3(fbits(x) & 0x7fffffffu, fbits(y) & 0x7fffffffu, fbits(z) & 0x7fffffffu) >= 0x7f800000u)
    return NormRound{0u, NORM_NONFINITE};
  int Emax = -1;
  for (int i = 0; i < 3; i++) {
    uint32_t u = fbits(c[i]) & 0x7fffffffu;
    uint32_t e = u >> 23, m = u & 0x7fffffu;
    if (e) m |= 0x800000u; else e = 1;
    Mf[i] = m;
    Ef[i] = e;
    if (m && (int)e > Emax) Emax = (int)e;
  }
  if (Emax < 0) return NormRound{0u, 0};
  // S in units of 2^(2 Emax - 300 - 64): term_i = Mf^2 << (2 (Ef - Emax) + 64)
  unsigned __int128 S = 0;
  bool sticky = false;
  for (int i = 0; i < 3; i++) {
    if (!Mf[i]) continue;
    unsigned __int128 sq = (unsigned __int128)((uint64_t)Mf[i] * (uint64_t)Mf[i]);
    int sh = 2 * ((int)Ef[i] - Emax) + 64;
    if (sh >= 0) S += sq << sh;
    else if (sh > -127) {
      unsigned __int128 lost = sq & ((((unsigned __int128)1) << (-sh)) - 1);
      sticky |= (lost != 0);
      S += sq >> (-sh);
    } else {
      sticky = true;
    }
  }
  // floor(log2 S) in absolute terms
  int bl;
  {
    uint64_t hi = (uint64_t)(S >> 64), lo = (uint64_t)S;
    bl = hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
  }
  const int unit = 2 * Emax - 364;                 // S_abs = S * 2^unit
  const int l2 = bl - 1 + unit;                    // floor(log2 S_abs)
  const int e_r = (l2 >= 0) ? l2 / 2 : -((-l2 + 1) / 2);   // floor(l2 / 2)
  int g = e_r - (prec - 1);
  if (keep_sub && g < -149) g = -149;
  // T4 = floor(4 S_abs / 4^g)
  const int sh = unit + 2 - 2 * g;
  uint64_t T4;
  if (sh >= 0) {
    T4 = (uint64_t)(S << sh);
  } else {
    const int rs = -sh;
    if (rs >= 128) { sticky |= (S != 0); T4 = 0; }
    else {
      unsigned __int128 lost = S & ((((unsigned __int128)1) << rs) - 1);
      sticky |= (lost != 0);
      T4 = (uint64_t)(S >> rs);
    }
  }
  // s = floor(sqrt(T4)), from a float estimate plus exact integer correction
  uint64_t s = (uint64_t)sqrtf((float)T4);
  while (s > 0 && s * s > T4) s--;
  while ((s + 1) * (s + 1) <= T4) s++;
  uint64_t j = s >> 1;
  const uint64_t m2 = (2 * j + 1) * (2 * j + 1);
  if (T4 > m2 || (T4 == m2 && sticky)) j += 1;
  else if (T4 == m2 && (j & 1)) j += 1;           // exact tie: to even
  if (j >> prec) { j >>= 1; g += 1; }             // carried into the next binade
  return NormRound{(uint32_t)j, g};
}

// Angle of (num, den), num, den >= 0 given as double-floats, as a level
// coordinate in double-float form:  V = B + s * C * atan(b) with the octant
// offsets B (multiples of K/4), so that  V = K * atan2(num, den)/(pi/2) * ...
// Concretely, with Kq = level count of a quarter turn (pi/2):
//   atan2(num, den) in [0, pi/2] maps to [0, Kq];  C = Kq/(pi/2) (double-float).
// Returns vh >= 0 and vl such that vh + vl = Kq * atan2(num, den)/(pi/2) when
// den_neg == false, and 2 Kq - that value when den_neg == true.
VC_DI void angle_levels(float num_h, float num_l, float den_h, float den_l, bool den_neg,
                        float Kq, float C_h, float C_l, float& vh, float& vl)
{
  constexpr float T8 = 0.41421356237309503f;      // tan(pi/8)
  const bool swap = num_h > den_h;
  const float mx_h = swap ? num_h : den_h, mx_l = swap ? num_l : den_l;
  const float mn_h = swap ? den_h : num_h, mn_l = swap ? den_l : num_l;
  const bool R = mn_h > T8 * mx_h;
  // reduced ratio b = mn/mx, or (mn - mx)/(mn + mx) with atan(a) = pi/4 + atan(b)
  const float d_h = mn_h - mx_h;                  // Fast2Sum, |mx| >= |mn|
  const float d_l = (mn_h - (d_h + mx_h)) + (mn_l - mx_l);
  const float s_h = mx_h + mn_h;
  const float s_l = (mn_h - (s_h - mx_h)) + (mn_l + mx_l);
  const float nu_h = R ? d_h : mn_h, nu_l = R ? d_l : mn_l;
  const float de_h = R ? s_h : mx_h, de_l = R ? s_l : mx_l;
  const float rc = rcp_(fmax_(de_h, 0x1p-120f));
  const float b0 = nu_h * rc;
  const float b1 = (fma_(-b0, de_h, nu_h) + (nu_l - b0 * de_l)) * rc;
  // atan(b) = b (1 + s R(s)), s = b^2
  const float s2 = b0 * b0;
  float Rp = VC_ATAN_R[VC_ATAN_R_DEG];
#pragma unroll
  for (int i = VC_ATAN_R_DEG - 1; i >= 0; i--) Rp = fma_(Rp, s2, VC_ATAN_R[i]);
  const float u = s2 * Rp;
  // L = C b (double-float), T = L u, H = L + T
  const float Lh = C_h * b0;
  const float Ll = fma_(C_h, b0, -Lh) + fma_(C_h, b1, C_l * b0);
  const float Tt = Lh * u;
  const float Hh = Lh + Tt;
  const float Hl = ((Lh - Hh) + Tt) + Ll;
  // octant offset in units of Kq/2: atan2 = [swap] pi/2 +- ([R] pi/4 + atan b), mirrored for den < 0
  const bool neg = den_neg != swap;
  const int k0 = swap ? 2 : (den_neg ? 4 : 0);
  const int kk = neg ? k0 - (int)R : k0 + (int)R;
  const float B = (float)kk * (0.5f * Kq);        // exact: a multiple of 1/8 below 2^18
  const float sg = neg ? -1.0f : 1.0f;
  const float sHh = sg * Hh, sHl = sg * Hl;
  // Fast2Sum: |B| >= |H| whenever B != 0
  vh = B + sHh;
  vl = (sHh - (vh - B)) + sHl;
}

// floor(vh + vl + c) for vh >= 0 (exact fraction), c a small exact constant
VC_DI int floor_dd(float vh, float vl, float c)
{
  const float k = floor_(vh);
  const float f = (vh - k) + (vl + c);
  return (int)k + (int)floor_(f);
}

// ceil(vh + vl + c) for vh >= 0
VC_DI int ceil_dd(float vh, float vl, float c)
{
  const float k = floor_(vh);
  const float f = (vh - k) + (vl + c);
  const float ff = floor_(f);
  return (int)k + (int)ff + (f != ff ? 1 : 0);
}

// Companding tail: h(u) = u (1 + w(u^2)); returns |Q| (1 + w) for |Q| = K |u| (double-float in/out)
template <int MODE>
VC_DI void compand_levels(float qh, float ql, float K, const Params& P, float& oh, float& ol)
{
  if (MODE == TANH) {
    const float u = qh * (1.0f / K);
    const float v = u * u;
    float acc = P.w[7];                          // degree 7 (the host fits P.w at that degree)
#pragma unroll
    for (int i = 6; i >= 0; i--) acc = fma_(acc, v, P.w[i]);
    const float d = qh * acc;                    // |Q| w, <= ~0.09 |Q|
    oh = qh + d;
    ol = ((qh - oh) + d) + ql * (1.0f + acc);
  } else {
    // cosine map: h(u) = sin(pi u/2).  Written as (pi/2) u - x^3/6 + x^5 P(x^2), x = pi u/2,
    // with the first two terms in double-float.
    const float PI2_h = 1.57079637f, PI2_l = -4.37113883e-08f;
    const float inv = 1.0f / K;
    // u = |Q|/K as double-float
    const float uh = qh * inv;
    const float ul = (fma_(-uh, K, qh) + ql) * inv;
    // x = (pi/2) u
    const float xh = PI2_h * uh;
    const float xl = fma_(PI2_h, uh, -xh) + (PI2_h * ul + PI2_l * uh);
    // x^2, x^3 double-float
    const float x2h = xh * xh;
    const float x2l = fma_(xh, xh, -x2h) + 2.0f * xh * xl;
    const float x3h = x2h * xh;
    const float x3l = fma_(x2h, xh, -x3h) + (x2h * xl + x2l * xh);
    // sin x = x - x^3/6 + x^5 (1/5! - x^2/7! + x^4/9! - x^6/11! + x^8/13! - x^10/15!)
    float t = -7.6471637e-13f;
    t = fma_(t, x2h, 1.6059044e-10f);
    t = fma_(t, x2h, -2.5052108e-08f);
    t = fma_(t, x2h, 2.7557319e-06f);
    t = fma_(t, x2h, -1.9841270e-04f);
    t = fma_(t, x2h, 8.3333333e-03f);
    const float x5t = x3h * x2h * t;
    const float sixth_h = 0.166666672f, sixth_l = -4.96705388e-09f;
    const float c3h = x3h * sixth_h;
    const float c3l = fma_(x3h, sixth_h, -c3h) + (x3l * sixth_h + x3h * sixth_l);
    // h = x - c3 + x5t (double-float)
    float sh = xh - c3h;
    float sl = ((xh - sh) - c3h) + (xl - c3l);    // |xh| >= |c3h|
    float th = sh + x5t;
    float tl = ((sh - th) + x5t) + sl;
    // levels: K h
    oh = K * th;
    ol = fma_(K, th, -oh) + K * tl;
  }
}

// ------------------------------------------------------------------ encode

// The companded level floor(K h(|Q| / K)) from an estimate f0 within one of it: the level is the
// number of boundaries T[1..] at or below |Q| (double-float qh + ql, not necessarily normalised),
// and h is increasing, so the signs of |Q| - T[f0] and |Q| - T[f0 + 1] settle it.  Entry f of the
// table (16 bytes, 16-byte aligned) holds T[f] and T[f + 1], high then low parts.  Each sign is
// taken from (qh - Th) + (ql - Tl): the first difference is exact whenever it is small (Sterbenz),
// so a wrong sign needs |Q| within ~2^-24 |ql| of the boundary; |Q| itself carries the encoder's
// error (about 2^-44 relative).  Both lie far inside the one-ulp window.
VC_DI int table_level(int f0, float qh, float ql, const float* T, int jmax)
{
  typedef float f32x4_t __attribute__((vector_size(16)));
  const int f = f0 < 0 ? 0 : (f0 > jmax ? jmax : f0);
  if (T == nullptr) return f;                       // (every encoding entry point attaches them)
  const f32x4_t e = *(const f32x4_t*)(T + 4 * f);
  const float db = (qh - e[0]) + (ql - e[1]);       // |Q| - (start of level f)
  const float dn = (qh - e[2]) + (ql - e[3]);       // |Q| - (start of level f + 1)
  // (|Q| cannot lie below the start of level f and at or past the start of level f + 1 at once)
  return (f > 0 && db < 0.0f) ? f - 1 : (dn >= 0.0f ? f + 1 : f);
}

// Code of a float32 vector (the compress function of §3), single-precision arithmetic only.
template <class L, int MODE>
VC_DI uint64_t encode_vec32(float x, float y, float z, const Params& P)
{
  const uint32_t ax = fbits(x) & 0x7fffffffu, ay = fbits(y) & 0x7fffffffu, az = fbits(z) & 0x7fffffffu;
  const uint32_t amax = umax3(ax, ay, az);
  if (amax >= 0x7f800000u) return L::reserved;    // non-finite input
  if (amax == 0u) return 0ull;                    // zero vector

  // ---- scale so that the largest component is in [0.5, 1) (exact)
  // amax = 1.f 2^(E-127) = 0.1f 2^(E-126): k = E - 126 (subnormal amax: k = -126)
  const int k = (int)(amax >> 23) - 126;
  const bool tiny = amax < 0x00800000u;           // all components subnormal: exact path only
  const float xs = ldexp_(x, -k), ys = ldexp_(y, -k), zs = ldexp_(z, -k);

  // ---- squares as double-floats
  const float px = xs * xs, py = ys * ys, pz = zs * zs;
  const float ex = fma_(xs, xs, -px), ey = fma_(ys, ys, -py), ez = fma_(zs, zs, -pz);
  // rho^2 = x^2 + y^2
  const float a1 = fmax_(px, py), b1 = fmin_(px, py);
  const float r2h = a1 + b1;
  const float r2l = (b1 - (r2h - a1)) + (ex + ey);
  // S = rho^2 + z^2 (TwoSum)
  const float Sh = r2h + pz;
  const float bb = Sh - r2h;
  const float Sl = ((r2h - (Sh - bb)) + (pz - bb)) + (r2l + ez);

  // ---- magnitude: r = sqrt(S) as r0 + rlo, then nearest-even at 1+mr bits
  const float rS = rsq_(Sh);
  const float r0 = Sh * rS;
  const float rlo = (fma_(-r0, r0, Sh) + Sl) * (0.5f * rS);
  const uint32_t b0 = fbits(r0);
  constexpr int drop = 23 - L::mr;                // grid step in ulps of r0 is 2^drop
  constexpr uint32_t lowm = (1u << drop) - 1u;
  const float v = ldexp_(rlo, 150 - (int)(b0 >> 23));   // rlo in ulps of r0
  const float pg = ((float)(b0 & lowm) + v) * (1.0f / (float)(1u << drop));
  const float fl = floor_(pg);
  const float fr = pg - fl;
  const uint32_t mant = b0 & 0x7fffffu;
  bool amb = (fabs_(fr - 0.5f) < 0x1p-14f) || (mant < 8u) || (mant > 0x7ffff7u) || tiny;
  const int jg = (int)fl + (fr > 0.5f ? 1 : 0);
  uint32_t rb = (b0 & ~lowm) + ((uint32_t)jg << drop);
  int e_r = (int)(rb >> 23) - 127 + k;            // unbiased exponent of r_hat
  uint32_t Mfield = (rb & 0x7fffffu) >> (23 - L::m);   // truncating: the low 23 - m bits drop
  if (L::keep_sub) amb = amb || (e_r + L::bias <= 1);
  if (amb) {
    uint32_t j;
    int g;
    const NormRound nr = exact_norm_round(x, y, z, L::mr + 1, L::keep_sub);
    j = nr.j;
    g = nr.g;
    if constexpr (L::trunc) { j >>= L::mr - L::m; g += L::mr - L::m; }
    if (j >= (1u << L::m)) {                      // normal
      e_r = g + L::m;
      Mfield = j - (1u << L::m);
    } else {                                      // subnormal (keep_sub only)
      e_r = -L::bias;                             // -> E = 0
      Mfield = j;
    }
  }
  int E = e_r + L::bias;
  if (E < 1 && !(L::keep_sub && E == 0)) return 0ull;   // underflow flushes to the zero code
  if (L::keep_sub && E == 0 && Mfield == 0u) return 0ull;
  if (E > L::emax) { E = L::emax; Mfield = (1u << L::m) - 1u; }   // saturate

  // ---- rho = sqrt(x^2 + y^2) as a double-float (for phi)
  const float rr = rsq_(fmax_(r2h, 0x1p-100f));
  const float rho_h = r2h * rr;
  const float rho_l = (fma_(-rho_h, rho_h, r2h) + r2l) * (0.5f * rr);

  // ---- theta = atan2(y, x) on |Q| = Kt |theta|/pi  (Kq = Kt/2 levels per quarter turn)
  float qh, ql;
  // signs from the unscaled inputs (a tiny component may underflow to -0 when scaled)
  const bool yneg = y < 0.0f, xneg = x < 0.0f, zneg = z < 0.0f;
  angle_levels(fabs_(ys), 0.0f, fabs_(xs), 0.0f, xneg, 0.5f * P.Kt, P.Ct_h, P.Ct_l, qh, ql);
  uint32_t nth;
  if ((MODE == TANH || MODE == COS) && P.comp_t) {
    // the companded level: an estimate from the single-precision map, settled by the table of
    // boundaries (odd n_theta_max: for y < 0 the level mirrors, base - 1 - f)
    float mh, ml;
    compand_levels<MODE>(qh, ql, P.Kt, P, mh, ml);
    const int f = table_level(floor_dd(mh, ml, 0.0f), qh, ql, P.ctab_t, (int)(P.nmax_t >> 1));
    nth = yneg ? (uint32_t)((int)P.base_t - 1 - f) : (uint32_t)((int)P.base_t + f);
  } else if (MODE == FRAC && !P.odd_t) {
    // even n_theta_max: n = n_max/2 + floor(Q + 1/2), Q = +-|Q|
    nth = yneg ? (uint32_t)((int)P.base_t - ceil_dd(qh, ql, -0.5f))
                      : (uint32_t)((int)P.base_t + floor_dd(qh, ql, 0.5f));
  } else {
    // odd n_theta_max: n = (n_max+1)/2 + floor(Q); for y < 0, |Q| is never an integer
    const int f = floor_dd(qh, ql, 0.0f);
    nth = yneg ? (uint32_t)((int)P.base_t - 1 - f) : (uint32_t)((int)P.base_t + f);
  }

  // ---- phi = atan2(rho, z): V = n_phi_max phi/pi + 1/2, n = floor(V)  (Kq = Np/2)
  float vh, vl;
  angle_levels(rho_h, rho_l, fabs_(zs), 0.0f, zneg, 0.5f * P.Np, P.Cp_h, P.Cp_l, vh, vl);
  uint32_t nph;
  if ((MODE == TANH || MODE == COS) && P.comp_p) {
    // centred coordinate Qc = V - 1/2 - Np/2 = (Np/2) u_phi; tie at phi = pi/2 (z == 0)
    const float Kc = 0.5f * P.Np;
    float ch = vh - Kc;                           // exact when vh in [Kc/2, 2 Kc]; else via Fast2Sum
    float cl;
    {
      const float big = fabs_(vh) >= Kc ? vh : -Kc, sml = fabs_(vh) >= Kc ? -Kc : vh;
      cl = (sml - (ch - big)) + vl;
    }
    const bool negc = ch < 0.0f || (ch == 0.0f && cl < 0.0f);
    const float ah = negc ? -ch : ch, al = negc ? -cl : cl;
    float mh, ml;
    compand_levels<MODE>(ah, al, Kc, P, mh, ml);
    const int base_p = (int)((P.nmax_p + 1u) / 2u);
    const int f = table_level(floor_dd(mh, ml, 0.0f), ah, al, P.ctab_p, (int)(P.nmax_p >> 1));
    nph = negc ? (uint32_t)(base_p - 1 - f) : (uint32_t)(base_p + f);
    if (z == 0.0f) nph = (uint32_t)base_p;
  } else {
    nph = (uint32_t)floor_dd(vh, vl, 0.5f);
  }

  // ---- pack: [s][E][M][n_phi][n_theta]  (Eq. q_split for the fractional split)
  uint64_t low;
  if (MODE == FRAC) low = (uint64_t)nph * (uint64_t)P.T + (uint64_t)nth;
  else low = ((uint64_t)nph << L::t) | (uint64_t)nth;
  return ((uint64_t)(uint32_t)E << L::sh_e) | ((uint64_t)Mfield << L::sh_m) | low;
}


// ------------------------------------------------------------------ FP64-assisted encode
// Same definitions, with the norm, the angle ratios and the level coordinates carried
// in double precision (the paper's implementation section prescribes double-precision
// intermediates for phi).  On gfx950 an FP64 FMA issues like an FP32 one, so this is
// cheaper than the double-float single-precision path.  The hardware FP64
// reciprocal/rsqrt are ~2^-24 accurate and get one correction step each.

// Level coordinate of an angle a in [0, pi] from the tangent of its half, t = num/den in [0, 1]
// (den > 0): a' = 2 atan(t) in [0, pi/2], and a = a' (reflect false) or pi - a' (reflect true).
// Kq is the level count of a quarter turn, so a = pi is 2 Kq levels, and C2 = 2 (2 Kq)/pi
// converts atan to levels.  Above t = tan(pi/8) the ratio is reduced, atan(t) = pi/4 +
// atan((num - den)/(num + den)), so the polynomial sees |b| <= tan(pi/8).  With V = [R] Kq +
// C2 atan(b) + add (add = 1/2 for HALF, else 0; the offsets are exact) the result is V, or
// 2 Kq + 2 add - V when reflected: |f (2 Kq + 2 add) - V| with f = 0 or 1, as V lies in
// [add, Kq + add].
template <bool HALF>
VC_DI double half_angle_levels64(double num, double den, bool reflect, double Kq, double C2)
{
  constexpr double add = HALF ? 0.5 : 0.0;
  constexpr double T8 = 0.41421356237309503;      // tan(pi/8)
  const bool R = num > T8 * den;
  // (nu, de) = R ? (num - den, num + den) : (num, den), as FMAs with a 0/1 factor (each one
  // rounding, or exact when the factor is 0)
  const double Rd = R ? 1.0 : 0.0;
  const double nu = fma64_(-Rd, den, num);
  const double de = fma64_(Rd, num, den);
  const double rc = rcp64_(de);
  double b = nu * rc;
  b = fma64_(fma64_(-b, de, nu), rc, b);          // quotient to ~2^-48
  const double s2 = b * b;
  double Rp = VC_ATAN_R64[VC_ATAN_R64_DEG];
#pragma unroll
  for (int i = VC_ATAN_R64_DEG - 1; i >= 0; i--) Rp = fma64_(Rp, s2, VC_ATAN_R64[i]);
  const double at = fma64_(b, s2 * Rp, b);        // atan(b)
  const double V = fma64_(C2, at, fma64_(Rd, Kq, add));
  const double f = reflect ? 1.0 : 0.0;
  return __builtin_fabs(fma64_(f, fma64_(2.0, Kq, 2.0 * add), -V));
}

// Companded level distance from the centre: K h(q/K) for q = K |u| >= 0.
template <int MODE, int TDEG = 15>
VC_DI double compand64(double q, double invK, const Params& P)
{
  const double u = q * invK;
  const double v = u * u;
  if (MODE == TANH) {
    // h(u)/u = W(u^2), fitted per gamma on the host to the degree it needs (at most 15, and at
    // most TDEG here; the coefficients above the fitted degree are zero)
    static_assert(TDEG >= 1 && TDEG <= 15, "tanh polynomial degree");
    double acc = P.w64[TDEG];
#pragma unroll
    for (int i = TDEG - 1; i >= 0; i--) acc = fma64_(acc, v, P.w64[i]);
    return q * acc;
  }
  // cosine map: h(u) = sin(pi u / 2) = (pi/2) u S(x^2), x = pi u / 2 (Taylor, |x| <= pi/2)
  const double x2 = 2.4674011002723395 * v;       // (pi/2)^2 u^2
  double t = -1.9572941063391263e-20;             // -1/21!
  t = fma64_(t, x2, 8.2206352466243295e-18);      //  1/19!
  t = fma64_(t, x2, -2.8114572543455206e-15);     // -1/17!
  t = fma64_(t, x2, 7.6471637318198164e-13);      //  1/15!
  t = fma64_(t, x2, -1.6059043836821613e-10);     // -1/13!
  t = fma64_(t, x2, 2.5052108385441720e-08);      //  1/11!
  t = fma64_(t, x2, -2.7557319223985888e-06);     // -1/9!
  t = fma64_(t, x2, 1.9841269841269841e-04);      //  1/7!
  t = fma64_(t, x2, -8.3333333333333332e-03);     // -1/5!
  t = fma64_(t, x2, 1.6666666666666666e-01);      //  1/3!
  const double S = fma64_(-t, x2, 1.0);
  return q * (1.5707963267948966 * S);
}

// Branch-free part of the FP64-assisted encoder: the code of (x, y, z), and `exact` set where the
// magnitude lies within 2^-44 of a rounding midpoint (or, for layouts that keep subnormals, in the
// lowest binade), where the code's E and M fields are to be replaced by encode64_exact_fix.  Every
// other case, non-finite input, underflow and saturation included, comes out final, by selects,
// so the only branch of encode_vec64 is the rare exact one.
template <class L, int MODE, int TDEG = 15>
VC_DI uint64_t encode_vec64_fast(float x, float y, float z, const Params& P, bool& slow)
{
  // |x|, |y|, |z| converted exactly; the squares are exact in FP64.  The signs come from the
  // inputs below.  A NaN in any component reaches r^2 and the non-finite test.
  const double X = (double)__builtin_fabsf(x), Y = (double)__builtin_fabsf(y), Z = (double)__builtin_fabsf(z);
  const double R2 = fma64_(X, X, Y * Y);          // rho^2, one rounding
  // r^2, two roundings (2^-52).  A finite float squares to below 2^256, so r^2 is finite exactly
  // when every component is.  The squares of nonzero floats are at least 2^-298, so adding
  // 2^-1000 to rho^2 changes only rho^2 = 0: r^2 changes only for the zero vector, whose norm
  // 2^-500 then flushes to the zero code like any norm under the smallest magnitude (through the
  // exact path).  For non-finite input the arithmetic below runs on infinities and NaNs and the
  // caller replaces its result with the reserved code.
  const double R2g = R2 + 0x1p-1000;              // == R2 unless R2 == 0
  const double S = fma64_(Z, Z, R2g);
  const bool bad = !(S < __builtin_huge_val());  // non-finite input (the test is false for NaN)

  // ---- magnitude: r to ~2^-47 (rsqrt seed + one Newton step), nearest-even at 1+mr bits
  const double yS = rsq64_(S);
  const double r0 = S * yS;
  const double r = fma64_(fma64_(-r0, r0, S), 0.5 * yS, r0);
  constexpr int drop = 52 - L::mr;                // fraction bits dropped from the FP64 value
  constexpr uint32_t half = 1u << (drop - 1);
  const uint64_t rb0 = dbits(r);
  const uint32_t low = (uint32_t)rb0 & ((1u << drop) - 1u);
  bool amb = (low - (half - 256u)) < 512u;        // within 2^-44 of a rounding midpoint
  // rounded, then (truncating layouts) the fraction bits below m dropped
  const uint64_t rb = (rb0 + half) & ~((1ull << (52 - L::m)) - 1ull);
  // code exponent E = e + bias lies in [1, emax]  <=>  rb in [rb_lo, rb_hi)
  constexpr uint64_t rb_lo = (uint64_t)(1024 - L::bias) << 52;
  constexpr uint64_t rb_hi = (uint64_t)(1024 - L::bias + L::emax) << 52;
  if (L::keep_sub) amb = amb || rb < rb_lo + (1ull << 52);   // E <= 1: subnormal codes, exact path
  // the slow path (the caller's): non-finite input, a norm near a rounding midpoint, and a code
  // exponent out of [1, emax] (underflow to the zero code, saturation), all decided there by the
  // exact norm
  slow = bad || amb || rb < rb_lo || rb >= rb_hi;
  // the FP64 exponent and fraction fields of rb moved to the code's E|M position, with the
  // exponent re-biased (modulo 2^64 the bits above the field drop out)
  constexpr int k = L::sh_e - 52;
  static_assert(k > 0, "code exponent field above bit 52");
  const uint64_t em = (rb << k) - ((uint64_t)(1023 - L::bias) << L::sh_e);

  // ---- rho = sqrt(x^2 + y^2) to ~2^-47, of R2g: 2^-500 on the z axis, so that the theta ratio
  //      below is 0 there; otherwise R2g == R2.  With z = 0, R2g == S, so this is the same
  //      computation on the same value as r above, and rho == r exactly there.
  const double yR = rsq64_(R2g);
  const double p0 = R2g * yR;
  const double rho = fma64_(fma64_(-p0, p0, R2g), 0.5 * yR, p0);

  // ---- theta: |Q| = Kt |theta|/pi; n = base + floor(+-|Q| (+1/2 if n_theta_max is even)).
  //      The half angle of |theta| in [0, pi] has the tangent |y| / (rho + x): from x >= 0,
  //      |y| / (rho + |x|) gives theta' = atan2(|y|, |x|), reflected (pi - theta') for x < 0.
  //      On the z axis (x = y = 0) rho = 2^-500, so the ratio is 0: theta = atan2(0, 0) = 0 (R12).
  const bool yneg = y < 0.0f, xneg = x < 0.0f, zneg = z < 0.0f;
  double Q = half_angle_levels64<false>(Y, rho + X, xneg, 0.5 * P.Kt64, 2.0 * P.Ct64);
  if ((MODE == TANH || MODE == COS) && P.comp_t) Q = compand64<MODE, TDEG>(Q, P.invKt64, P);
  Q = level_guard(Q);
  uint32_t nth;
  if (MODE == FRAC) {
    const double Qs = yneg ? -Q : Q;
    nth = (uint32_t)((int)P.base_t + (int)floor64_(P.odd_t ? Qs : Qs + 0.5));
  } else {
    // n_theta_max odd: for y < 0, |Q| is never an integer, so floor(-|Q|) = -1 - floor(|Q|);
    // |Q| >= 0, so the truncating conversion is the floor
    const int f = (int)Q;
    nth = yneg ? (uint32_t)((int)P.base_t - 1 - f) : (uint32_t)((int)P.base_t + f);
  }

  // ---- phi: V = n_phi_max phi/pi; n = floor(V + 1/2).  The half angle of phi' = atan2(rho, |z|)
  //      has the tangent rho / (r + |z|) in [0, 1] (r + |z| >= r > 0); phi = pi - phi' for z < 0.
  //      At z = 0, rho == r, so the ratio is exactly 1 and phi exactly pi/2 (the tie of R3).
  uint32_t nph;
  if ((MODE == TANH || MODE == COS) && P.comp_p) {
    const double V = half_angle_levels64<false>(rho, r + Z, zneg, 0.5 * P.Np64, 2.0 * P.Cp64);
    const double Qc = V - 0.5 * P.Np64;           // (n_phi_max/2) u_phi, exact zero at phi = pi/2
    const double m = level_guard(compand64<MODE, TDEG>(__builtin_fabs(Qc), P.invKc64, P));
    nph = (uint32_t)((int)((P.nmax_p + 1u) / 2u) + (int)floor64_(Qc < 0 ? -m : m));
  } else {
    const double Vh = level_guard(half_angle_levels64<true>(rho, r + Z, zneg, 0.5 * P.Np64, 2.0 * P.Cp64));   // V + 1/2
    nph = (uint32_t)(int)Vh;                      // Vh >= 0: truncation is the floor
  }

  uint64_t w;
  if (MODE == FRAC) {
    w = em | ((uint64_t)nph * (uint64_t)P.T + (uint64_t)nth);
  } else {
    // the E and M fields lie in the high word; n_phi straddles the two words
    const uint32_t lo = nth | (nph << L::t);
    const uint32_t hi = (uint32_t)(em >> 32) | (nph >> (32 - L::t));
    w = ((uint64_t)hi << 32) | lo;
  }
  return w;
}

// The code's E and M fields from the exact norm (nearest-even at 1+mr bits, decided by integer
// arithmetic), merged with the angle fields of `w` (a code of the same vector): the cases
// encode_vec64_fast leaves to the slow path.  Underflow gives the zero code, overflow saturates,
// non-finite input gives the reserved code.
template <class L>
VC_DI uint64_t encode64_exact_fix(float x, float y, float z, uint64_t w)
{
  uint32_t j;
  int g, e_r;
  uint32_t Mfield;
  const NormRound nr = exact_norm_round(x, y, z, L::mr + 1, L::keep_sub);
  if (nr.g == NORM_NONFINITE) return L::reserved;
  j = nr.j;
  g = nr.g;
  if constexpr (L::trunc) { j >>= L::mr - L::m; g += L::mr - L::m; }
  if (j >= (1u << L::m)) { e_r = g + L::m; Mfield = j - (1u << L::m); }
  else { e_r = -L::bias; Mfield = j; }
  const int E = e_r + L::bias;
  if (E < 1 && !(L::keep_sub && E == 0)) return 0ull;   // underflow flushes to the zero code
  if (L::keep_sub && E == 0 && Mfield == 0u) return 0ull;
  const uint64_t em = E > L::emax ? L::saturated                        // saturate, angles kept
                                  : ((uint64_t)(uint32_t)E << L::sh_e) | ((uint64_t)Mfield << L::sh_m);
  return (w & ((1ull << L::sh_m) - 1ull)) | em;
}

template <class L, int MODE, int TDEG = 15>
VC_DI uint64_t encode_vec64(float x, float y, float z, const Params& P)
{
  bool slow;
  const uint64_t w = encode_vec64_fast<L, MODE, TDEG>(x, y, z, P, slow);
  return slow ? encode64_exact_fix<L>(x, y, z, w) : w;
}

// precision dispatch
template <class L, int MODE, int PREC, int TDEG = 15>
VC_DI uint64_t encode_vec(float x, float y, float z, const Params& P)
{
  if constexpr (PREC == PREC_F64) return encode_vec64<L, MODE, TDEG>(x, y, z, P);
  else return encode_vec32<L, MODE>(x, y, z, P);
}

}  // namespace vc
