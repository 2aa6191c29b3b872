// vc_params.hpp -- host-side resolution of a vc_codec into the kernels' constants.
// Host-only C++ (no device code); included by the C ABI and by the CPU emulation
// build of the codec.
#pragma once

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/vc.h"
#include "../../include/vc_device.hpp"

namespace vc {

// Resolved codec: compile-time layout/mode ids plus the runtime constants.
struct Resolved {
  int layout;      // vc_layout
  int mode;        // vc::Mode
  int mag_round;   // vc_mag_round
  int prec;        // vc::Prec
  Params P;
};

static const struct {
  const char* name;
  int layout;
} kLayouts[] = {
    {"0,7,22-17-18", VC_LAYOUT_0_7_22_17_18},
    {"0,7,23-17-17", VC_LAYOUT_0_7_23_17_17},
    {"0,8,23-16-17", VC_LAYOUT_0_8_23_16_17},
    {"1,8,23-16-16", VC_LAYOUT_1_8_23_16_16},
};

struct LayoutBits {
  int e, m, p, t, bias;
};
static inline LayoutBits layout_bits(int layout)
{
  switch (layout) {
    case VC_LAYOUT_0_7_22_17_18: return {7, 22, 17, 18, 80};
    case VC_LAYOUT_0_7_23_17_17: return {7, 23, 17, 17, 80};
    case VC_LAYOUT_0_8_23_16_17: return {8, 23, 16, 17, 127};
    default: return {8, 23, 16, 16, 127};
  }
}

static inline void split_dd(long double v, float* hi, float* lo)
{
  float h = (float)v;
  *hi = h;
  *lo = (float)(v - (long double)h);
}

// Least-squares fit (Chebyshev nodes) of w(v) = tanh(gamma sqrt v)/(tanh(gamma) sqrt v) - 1 on
// v in [0, 1]; returns the max residual of the float32 coefficients.
static inline double fit_tanh_tail(double gamma, float* w, int deg)
{
  const int N = 400;
  const int D = deg + 1;
  long double A[16][16] = {{0}}, rhs[16] = {0};
  const long double c = tanhl((long double)gamma);
  for (int k = 0; k < N; k++) {
    long double v = 0.5L + 0.5L * cosl(3.14159265358979323846264338327950288L * (k + 0.5L) / N);
    long double u = sqrtl(v);
    long double f = (u < 1e-6L) ? (gamma / c) * (1.0L - gamma * gamma * v / 3.0L) - 1.0L
                                : tanhl(gamma * u) / (c * u) - 1.0L;
    long double pw[16];
    pw[0] = 1.0L;
    for (int i = 1; i < D; i++) pw[i] = pw[i - 1] * v;
    for (int i = 0; i < D; i++) {
      rhs[i] += pw[i] * f;
      for (int j = 0; j < D; j++) A[i][j] += pw[i] * pw[j];
    }
  }
  // Gaussian elimination with partial pivoting
  for (int i = 0; i < D; i++) {
    int piv = i;
    for (int r = i + 1; r < D; r++)
      if (fabsl(A[r][i]) > fabsl(A[piv][i])) piv = r;
    for (int j = 0; j < D; j++) { long double t = A[i][j]; A[i][j] = A[piv][j]; A[piv][j] = t; }
    { long double t = rhs[i]; rhs[i] = rhs[piv]; rhs[piv] = t; }
    for (int r = i + 1; r < D; r++) {
      long double f = A[r][i] / A[i][i];
      for (int j = i; j < D; j++) A[r][j] -= f * A[i][j];
      rhs[r] -= f * rhs[i];
    }
  }
  long double coef[16];
  for (int i = D - 1; i >= 0; i--) {
    long double s = rhs[i];
    for (int j = i + 1; j < D; j++) s -= A[i][j] * coef[j];
    coef[i] = s / A[i][i];
  }
  for (int i = 0; i < D; i++) w[i] = (float)coef[i];
  double maxerr = 0.0;
  for (int k = 0; k <= 2000; k++) {
    double u = k / 2000.0, v = u * u;
    double f = (u < 1e-6) ? (gamma / (double)c) - 1.0 : tanh(gamma * u) / ((double)c * u) - 1.0;
    double acc = w[deg];
    for (int i = deg - 1; i >= 0; i--) acc = acc * v + w[i];
    double e = fabs(acc - f);
    if (e > maxerr) maxerr = e;
  }
  return maxerr;
}

// W(v) = tanh(gamma sqrt v)/(tanh(gamma) sqrt v) on v in [0, 1]: h(u)/u of the tanh
// companding map (u^2 = v).
static inline long double tanh_ratio(long double gamma, long double v)
{
  const long double c = tanhl(gamma);
  const long double u = sqrtl(v);
  if (u < 1e-7L) return gamma / c * (1.0L - gamma * gamma * v / 3.0L);
  return tanhl(gamma * u) / (c * u);
}

// Chebyshev projection of W on [0, 1] (128 nodes, long double), truncated at `deg` and
// converted to monomial coefficients in v.  Returns the max residual of the double
// coefficients on a fine grid.
static inline double fit_tanh_ratio64(double gamma, double* w, int deg)
{
  const int M = 128;
  long double a[20] = {0};
  for (int k = 0; k <= deg; k++) {
    long double sacc = 0.0L;
    for (int j = 0; j < M; j++) {
      const long double th = 3.14159265358979323846264338327950288L * (j + 0.5L) / M;
      const long double t = cosl(th);
      sacc += tanh_ratio(gamma, 0.5L * (t + 1.0L)) * cosl(k * th);
    }
    a[k] = sacc * 2.0L / M;
  }
  a[0] *= 0.5L;
  // sum a_k T_k(t), t = 2v - 1  ->  monomials in v
  long double Tkm1[20] = {0}, Tk[20] = {0}, Tkp1[20], mono[20] = {0};
  Tkm1[0] = 1.0L;                       // T_0 = 1
  Tk[0] = -1.0L; Tk[1] = 2.0L;          // T_1 = 2v - 1
  for (int i = 0; i <= deg; i++) mono[i] += a[0] * Tkm1[i];
  if (deg >= 1) for (int i = 0; i <= deg; i++) mono[i] += a[1] * Tk[i];
  for (int k = 2; k <= deg; k++) {
    // T_{k} = 2 t T_{k-1} - T_{k-2} = (4v - 2) T_{k-1} - T_{k-2}
    for (int i = 0; i <= deg; i++) {
      long double vprev = i ? Tk[i - 1] : 0.0L;
      Tkp1[i] = 4.0L * vprev - 2.0L * Tk[i] - Tkm1[i];
    }
    for (int i = 0; i <= deg; i++) { Tkm1[i] = Tk[i]; Tk[i] = Tkp1[i]; }
    for (int i = 0; i <= deg; i++) mono[i] += a[k] * Tk[i];
  }
  for (int i = 0; i <= deg; i++) w[i] = (double)mono[i];
  double maxerr = 0.0;
  for (int k = 0; k <= 4000; k++) {
    const long double u = k / 4000.0L, v = u * u;
    long double acc = w[deg];
    for (int i = deg - 1; i >= 0; i--) acc = acc * v + w[i];
    const double e = (double)fabsl(acc - tanh_ratio(gamma, v));
    if (e > maxerr) maxerr = e;
  }
  return maxerr;
}

// The tanh map's polynomial fits depend on gamma alone and take milliseconds of host time, while
// resolve() runs on every library call: they are cached per gamma (a small table under a lock;
// past 16 distinct values the oldest entry is replaced).
static inline vc_status tanh_fits(float gamma, Params& P)
{
  struct Entry {
    uint32_t gamma_bits;
    vc_status st;
    float w[8];
    int wdeg64;
    double w64[16];
  };
  static std::mutex mu;
  static Entry table[16];
  static int used = 0, next = 0;
  uint32_t gb;
  memcpy(&gb, &gamma, sizeof gb);
  std::lock_guard<std::mutex> lk(mu);
  for (int i = 0; i < used; i++) {
    if (table[i].gamma_bits == gb) {
      memcpy(P.w, table[i].w, sizeof P.w);
      P.wdeg = 7;
      P.wdeg64 = table[i].wdeg64;
      memcpy(P.w64, table[i].w64, sizeof P.w64);
      return table[i].st;
    }
  }
  Entry e;
  memset(&e, 0, sizeof e);
  e.gamma_bits = gb;
  e.st = VC_SUCCESS;
  const double err = fit_tanh_tail((double)gamma, e.w, 7);
  if (err > 2e-8) e.st = VC_ERROR_UNSUPPORTED_CODEC;   // residual relative to |Q| scales like the 1-ulp window
  // smallest degree whose double-precision fit is within 1e-14 (the level error near the
  // phi poles is Kc times this residual)
  double err64 = 1.0;
  for (e.wdeg64 = 6; e.wdeg64 <= 15; e.wdeg64++) {
    memset(e.w64, 0, sizeof e.w64);
    err64 = fit_tanh_ratio64((double)gamma, e.w64, e.wdeg64);
    if (err64 <= 1e-14) break;
  }
  if (err64 > 1e-14) e.st = VC_ERROR_UNSUPPORTED_CODEC;
  Entry& slot = used < 16 ? table[used++] : table[next++ % 16];
  slot = e;
  memcpy(P.w, e.w, sizeof P.w);
  P.wdeg = 7;
  P.wdeg64 = e.wdeg64;
  memcpy(P.w64, e.w64, sizeof P.w64);
  return e.st;
}

// Level boundaries of a companded angle for the single-precision encoder: T[j] = K h^-1(j / K)
// in the uniform level coordinate |Q| (j = 1 .. floor(K)), T[0] = 0 and a last entry past every
// |Q|, each as a double-float pair.  h^-1 is atanh(v tanh g) / g (tanh map, R17) or
// (2/pi) asin(v) (cosine map, R18), in long double.  The table handed to the encoder holds one
// 16-byte entry per level f (T[f] and T[f + 1], high then low parts), so that one aligned load
// settles a level.
static inline void compand_boundaries(int mode, float gamma, double K, std::vector<float>& Q)
{
  const int jmax = (int)floor(K);
  std::vector<float> T(2 * (size_t)(jmax + 2), 0.0f);
  const long double PI = 3.14159265358979323846264338327950288L;
  const long double g = gamma, tg = tanhl(g);
  for (int j = 1; j <= jmax; j++) {
    const long double v = (long double)j / (long double)K;
    const long double u = mode == VC_MODE_TANH ? atanhl(v * tg) / g : (2.0L / PI) * asinl(v);
    split_dd((long double)K * u, &T[2 * (size_t)j], &T[2 * (size_t)j + 1]);
  }
  T[2 * (size_t)(jmax + 1)] = 3.0e38f;
  T[2 * (size_t)(jmax + 1) + 1] = 0.0f;
  // one 16-byte entry per level f = 0 .. jmax: the boundaries at its start and at its end
  Q.resize(4 * (size_t)(jmax + 1));
  for (size_t f = 0; f <= (size_t)jmax; f++)
    for (int i = 0; i < 4; i++) Q[4 * f + i] = T[2 * f + i];
}

// The boundary tables of (mode, gamma) for theta and phi of the default layout, built once per
// codec and device and kept until the process ends (up to 16 codecs; the GPU copies are made on
// the current device).  Only the single-precision encoder of a companded codec uses them.
static inline vc_status compand_tables(int mode, float gamma, const float** tt, const float** tp)
{
  struct Entry {
    int mode, dev;
    uint32_t gamma_bits;
    const float* t;
    const float* p;
  };
  static std::mutex mu;
  static Entry table[16];
  static int used = 0;
  uint32_t gb;
  memcpy(&gb, &gamma, sizeof gb);
  if (mode == VC_MODE_COS) gb = 0;                 // the cosine map has no parameter
  int dev = 0;
#ifndef VC_HOST_EMULATION
  if (hipGetDevice(&dev) != hipSuccess) return VC_ERROR_HIP;
#endif
  std::lock_guard<std::mutex> lk(mu);
  for (int i = 0; i < used; i++)
    if (table[i].mode == mode && table[i].gamma_bits == gb && table[i].dev == dev) {
      *tt = table[i].t;
      *tp = table[i].p;
      return VC_SUCCESS;
    }
  if (used == 16) return VC_ERROR_UNSUPPORTED_CODEC;
  // the default layout's level counts (companding is built for <0,7,22>-17-18 only)
  std::vector<float> ht, hp;
  compand_boundaries(mode, gamma, ((1 << 18) - 1) / 2.0, ht);
  compand_boundaries(mode, gamma, ((1 << 17) - 1) / 2.0, hp);
  const float *t = nullptr, *p = nullptr;
#ifdef VC_HOST_EMULATION
  // 16-byte aligned, as the device copies (an entry is read as one 16-byte vector)
  float* ht_own = static_cast<float*>(aligned_alloc(16, ht.size() * sizeof(float)));
  float* hp_own = static_cast<float*>(aligned_alloc(16, hp.size() * sizeof(float)));
  if (ht_own == nullptr || hp_own == nullptr) {
    free(ht_own);
    free(hp_own);
    return VC_ERROR_OUT_OF_MEMORY;
  }
  memcpy(ht_own, ht.data(), ht.size() * sizeof(float));
  memcpy(hp_own, hp.data(), hp.size() * sizeof(float));
  t = ht_own;
  p = hp_own;
#else
  float *dt = nullptr, *dp = nullptr;
  if (hipMalloc((void**)&dt, ht.size() * sizeof(float)) != hipSuccess) return VC_ERROR_OUT_OF_MEMORY;
  if (hipMalloc((void**)&dp, hp.size() * sizeof(float)) != hipSuccess) {
    (void)hipFree(dt);
    return VC_ERROR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(dt, ht.data(), ht.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dp, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dt);
    (void)hipFree(dp);
    return VC_ERROR_HIP;
  }
  t = dt;
  p = dp;
#endif
  table[used++] = Entry{mode, dev, gb, t, p};
  *tt = t;
  *tp = p;
  return VC_SUCCESS;
}

inline vc_status resolve(const vc_codec* c, Resolved* R)
{
  if (!c || !R) return VC_ERROR_INVALID_VALUE;
  if (c->struct_size != sizeof(vc_codec)) return VC_ERROR_INVALID_VALUE;
  if (c->layout > VC_LAYOUT_1_8_23_16_16) return VC_ERROR_UNSUPPORTED_CODEC;
  if (c->mode > VC_MODE_FRACSPLIT) return VC_ERROR_UNSUPPORTED_CODEC;
  if (c->mag_round > VC_MAG_TRUNC) return VC_ERROR_UNSUPPORTED_CODEC;
  if (c->precision > VC_PREC_F32 || c->reserved0 != 0) return VC_ERROR_INVALID_VALUE;
  if (c->mode != VC_MODE_PLAIN && c->layout != VC_LAYOUT_0_7_22_17_18) return VC_ERROR_UNSUPPORTED_CODEC;
  memset(R, 0, sizeof(*R));
  R->layout = (int)c->layout;
  R->mode = (int)c->mode;
  // with a 23-bit mantissa the truncation drops no bits: the magnitude is the float32 norm, which
  // nearest-even at 24 bits gives as well (on the float32 subnormal grid where the layout keeps
  // subnormals; a float32 overflow and an exponent above the field's both saturate)
  R->mag_round = (c->mag_round == VC_MAG_TRUNC && layout_bits((int)c->layout).m < 23) ? VC_MAG_TRUNC
                                                                                      : VC_MAG_RNE;
  R->prec = c->precision == VC_PREC_F32 ? PREC_F32 : PREC_F64;
  Params& P = R->P;
  const LayoutBits lb = layout_bits((int)c->layout);
  uint64_t nt, np;
  if (c->mode == VC_MODE_FRACSPLIT) {
    const uint64_t cap = 1ull << (lb.p + lb.t);
    if (c->frac_P < 2 || c->frac_P >= cap / 2) return VC_ERROR_INVALID_VALUE;
    const uint64_t T = cap / c->frac_P;        // largest T with P T <= 2^(p+t)  (Eq. q_split)
    if (T < 2 || T > (1ull << 24) || c->frac_P > (1ull << 24)) return VC_ERROR_UNSUPPORTED_CODEC;
    nt = T - 1;
    np = c->frac_P - 1;
    P.T = (uint32_t)T;
    P.limit = c->frac_P * T;
    P.invT64 = 1.0 / (double)T;
  } else {
    nt = (1ull << lb.t) - 1;
    np = (1ull << lb.p) - 1;
    P.T = (uint32_t)(nt + 1);
    P.limit = ~0ull;
  }
  P.nmax_t = (uint32_t)nt;
  P.nmax_p = (uint32_t)np;
  P.odd_t = (uint32_t)(nt & 1);
  P.base_t = (uint32_t)((nt & 1) ? (nt + 1) / 2 : nt / 2);
  P.Kt = (float)((double)nt / 2.0);
  P.Np = (float)np;
  P.half_t = P.Kt;
  const long double PI = 3.14159265358979323846264338327950288L;
  split_dd((long double)nt / 2.0L / PI, &P.Ct_h, &P.Ct_l);
  split_dd((long double)np / PI, &P.Cp_h, &P.Cp_l);
  split_dd(1.0L / (long double)nt, &P.rt_h, &P.rt_l);
  split_dd(1.0L / (2.0L * (long double)np), &P.rp_h, &P.rp_l);
  P.Kt64 = (double)nt / 2.0;
  P.Np64 = (double)np;
  P.Ct64 = (double)((long double)nt / 2.0L / PI);
  P.Cp64 = (double)((long double)np / PI);
  P.invKt64 = (double)(2.0L / (long double)nt);
  P.invKc64 = (double)(2.0L / (long double)np);
  if (c->mode == VC_MODE_TANH || c->mode == VC_MODE_COS) {
    P.comp_t = (c->compand_mask & VC_COMPAND_THETA) ? 1u : 0u;
    P.comp_p = (c->compand_mask & VC_COMPAND_PHI) ? 1u : 0u;
  }
  if (c->mode == VC_MODE_TANH) {
    if (!(c->gamma > 0.0f) || c->gamma > 1.0f) return VC_ERROR_UNSUPPORTED_CODEC;
    P.gam = c->gamma;
    P.inv_gam = 1.0f / c->gamma;
    P.cgam = (float)tanh((double)c->gamma);
    const vc_status fst = tanh_fits(c->gamma, P);
    if (fst != VC_SUCCESS) return fst;
  }
  return VC_SUCCESS;
}

// The boundary tables of a resolved codec whose single-precision encoder compands (no-op for
// every other codec): called by the entry points that encode, after their argument checks, so
// that validation-only calls (n == 0) and the decode-only paths allocate nothing.
inline vc_status attach_tables(const vc_codec* c, Resolved* R)
{
  if (R->prec == PREC_F32 && (R->mode == VC_MODE_TANH || R->mode == VC_MODE_COS))
    return compand_tables(R->mode, c->gamma, &R->P.ctab_t, &R->P.ctab_p);
  return VC_SUCCESS;
}

}  // namespace vc
