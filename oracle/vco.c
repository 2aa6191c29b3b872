/*
 * vco.c -- CPU oracle for the inline 3-vector compression of Trojak & Witherden
 * (arXiv 2003.02633).  TEST INFRASTRUCTURE ONLY: see vco.h.
 *
 * Each step follows the paper's definitions in its own notation:
 *   - spherical coordinates r, theta, phi of a Cartesian vector      §2.1, Eqs. (cart2sphere, spherical)
 *   - uniform angle quantisation with round-half-up nint()            §2.1, Eq. (a_disc) and the nint definition
 *   - inverse map of the levels back to angles                        §2.1, Eq. (a_inv)
 *   - magnitude with a shortened exponent (bias b_7) and mantissa     §2.3
 *   - bit layout <s,e,m>-p-t, fields MSB->LSB: sign, exponent,
 *     mantissa, n_phi, n_theta                                        §2.3, Fig. (comp_regimes)
 *   - fractional splitting n_p = n_phi (n_theta_max + 1) + n_theta    §2.4, Eq. (q_split)
 *   - tanh and cosine companding maps                                 §2.5
 *
 * Readings of points where the paper is silent or ambiguous are marked
 * "reading:" below.
 *
 * Arithmetic is FP64 and integer.  The only places where FP64 rounding could
 * change an integer decision are (a) the magnitude, which the paper defines as
 * a rounding of the exact norm, decided here exactly with expansion arithmetic,
 * and (b) level coordinates within ~1e-16 of a boundary, which is far inside the
 * one-ulp-of-single-precision window the GPU comparison allows.
 */
#include "vco.h"
#include <math.h>
#include <float.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* RN64(pi).  Dividing atan2() (which returns RN64 values of the exact angles at
 * multiples of pi/4) by this constant makes the half-revolution coordinate of
 * the axis directions exactly 0, 1/4, 1/2, 1; the exact-real ties of the
 * round-half-up rule (theta = 0, phi = pi/2) are then reproduced exactly. */
static const double PI64 = 3.141592653589793115997963468544185161590576171875;

/* ------------------------------------------------------------------------- */
/* exact helpers                                                              */
/* ------------------------------------------------------------------------- */

/* Knuth's TwoSum: s + e == a + b exactly. */
static void two_sum(double a, double b, double* s, double* e)
{
  double x = a + b;
  double bb = x - a;
  *e = (a - (x - bb)) + (b - bb);
  *s = x;
}

/* Sign of an exact sum of doubles by growing a nonoverlapping expansion
 * (Shewchuk 1997, Grow-Expansion with zero elimination).  The largest
 * component of a nonoverlapping expansion carries the sign of the sum. */
int vco_exact_sign(const double* v, int n)
{
  double e[32];
  int m = 0;
  if (n > 30) return 2; /* refuse: caller error */
  for (int i = 0; i < n; i++) {
    double q = v[i];
    int k = 0;
    for (int j = 0; j < m; j++) {
      double s, err;
      two_sum(q, e[j], &s, &err);
      if (err != 0.0) e[k++] = err;
      q = s;
    }
    if (q != 0.0) e[k++] = q;
    m = k;
  }
  if (m == 0) return 0;
  return e[m - 1] > 0.0 ? 1 : -1;
}

/* Round the exact Euclidean norm sqrt(x^2+y^2+z^2) of three singles to `prec`
 * significant bits, ties to even.  Below the normal range the grid spacing is
 * `min_spacing` when it is positive (gradual underflow); otherwise the
 * precision-relative grid is used at every magnitude.
 *
 * Method: FP64 gives the norm to ~1e-16, which fixes the binade and the
 * rounding midpoint `mid` between the two candidate grid values; whether the
 * exact norm lies above, below or on `mid` is the sign of
 * x^2 + y^2 + z^2 - mid^2, each term exact in FP64, summed exactly. */
double vco_round_norm(float x, float y, float z, int prec, double min_spacing, int* tie)
{
  double X2 = (double)x * (double)x;
  double Y2 = (double)y * (double)y;
  double Z2 = (double)z * (double)z;
  double S = X2 + Y2 + Z2;
  if (tie) *tie = 0;
  if (S == 0.0) return 0.0;
  double r = sqrt(S);
  int ex;
  (void)frexp(r, &ex);              /* r = f 2^ex, f in [0.5, 1) */
  int e = ex - 1;                   /* r in [2^e, 2^(e+1)) */
  double u = ldexp(1.0, e - (prec - 1));
  if (min_spacing > 0.0 && u < min_spacing) u = min_spacing;
  double k = floor(r / u) * u;      /* grid value at or below r */
  double mid = k + 0.5 * u;         /* <= prec+1 significant bits */
  double v[4] = {X2, Y2, Z2, -(mid * mid)};   /* mid*mid exact: <= 2*(prec+1) <= 52 bits */
  int sg = vco_exact_sign(v, 4);
  if (sg > 0) return k + u;
  if (sg < 0) return k;
  if (tie) *tie = 1;
  return (fmod(k / u, 2.0) == 0.0) ? k : k + u;
}

/* Single-precision result of alpha*a + b with exactly one rounding, i.e. the
 * value an IEEE fused multiply-add in binary32 returns.  alpha*a is exact in
 * FP64; the sum is kept as an unevaluated pair (s, err) and rounded once. */
float vco_rn32_fma(float alpha, float a, float b)
{
  double p = (double)alpha * (double)a;
  double s, err;
  two_sum(p, (double)b, &s, &err);
  if (!isfinite(s)) return (float)s;
  float f = (float)s;
  if (err == 0.0 || (double)f == s || !isfinite(f)) return f;
  /* s is not a float: the only way RN32(s) != RN32(s + err) is that s sits
   * exactly on the midpoint of two adjacent floats. */
  float g = nextafterf(f, (double)f < s ? INFINITY : -INFINITY);
  double mid = 0.5 * ((double)f + (double)g);
  if (s != mid) return f;
  if (err > 0.0) return fmaxf(f, g);
  return fminf(f, g);
}

static double ulp32_of(double v)
{
  v = fabs(v);
  if (v == 0.0 || v < 0x1p-126) return 0x1p-149;
  int e = ilogb(v);
  return ldexp(1.0, e - 23);
}

/* ------------------------------------------------------------------------- */
/* parameters                                                                 */
/* ------------------------------------------------------------------------- */

int vco_check(const vco_codec* c)
{
  if (!c) return 1;
  if (c->s < 0 || c->s > 1) return 2;
  if (c->e < 2 || c->e > 8) return 3;
  if (c->m < 1 || c->m > 23) return 4;
  if (c->p < 1 || c->t < 1 || c->p > 32 || c->t > 32) return 5;
  if (c->s + c->e + c->m + c->p + c->t > 64) return 6;
  if (c->mode < VCO_PLAIN || c->mode > VCO_FRAC) return 7;
  if (c->mode == VCO_FRAC) {
    uint64_t cap = 1ULL << (c->p + c->t);
    if (c->P < 2 || c->P >= cap / 2) return 8;
  }
  if (c->mode == VCO_TANH && !(c->gamma > 0.0)) return 9;
  return 0;
}

uint64_t vco_frac_T(const vco_codec* c)
{
  /* reading: the largest n_theta_max + 1 = T with P*T <= 2^(p+t), Eq. (q_split) */
  return (1ULL << (c->p + c->t)) / c->P;
}

uint64_t vco_nmax_theta(const vco_codec* c)
{
  if (c->mode == VCO_FRAC) return vco_frac_T(c) - 1;
  return (1ULL << c->t) - 1;   /* maximum of a t-bit unsigned integer, §2.1 */
}

uint64_t vco_nmax_phi(const vco_codec* c)
{
  if (c->mode == VCO_FRAC) return c->P - 1;
  return (1ULL << c->p) - 1;
}

static int keeps_subnormals(const vco_codec* c)
{
  /* reading: with the unchanged IEEE exponent (e = 8, b = 127) the magnitude
   * field is the single-precision value itself, gradual underflow included. */
  return c->e == 8 && c->bias == 127;
}

static int companded(const vco_codec* c, int is_theta)
{
  if (c->mode != VCO_TANH && c->mode != VCO_COS) return 0;
  return is_theta ? (c->compand_mask & VCO_COMP_THETA) != 0 : (c->compand_mask & VCO_COMP_PHI) != 0;
}

/* ------------------------------------------------------------------------- */
/* angle maps                                                                 */
/*                                                                            */
/* Both angles are written on a signed normalised coordinate u in [-1, 1]:    */
/*   theta: u = theta/pi            (psi = (theta + pi)/(2 pi) = (u+1)/2)      */
/*   phi:   u = 2 phi/pi - 1        (psi = phi/pi = (u+1)/2)                   */
/* The paper's maps n = nint(n_max f(psi)) become n = nint(n_max (1+h(u))/2): */
/*   plain (Eq. a_disc):   h(u) = u                                           */
/*   tanh  (§2.5):         h(u) = tanh(gamma u)/tanh(gamma)                   */
/*   cosine (§2.5):        1 - cos(pi psi) = 1 + sin(pi u/2), h(u) = sin(pi u/2)*/
/* ------------------------------------------------------------------------- */

static double hmap(const vco_codec* c, int is_theta, double u)
{
  if (!companded(c, is_theta)) return u;
  if (c->mode == VCO_TANH) return tanh(c->gamma * u) / tanh(c->gamma);
  return sin(0.5 * PI64 * u);
}

static double hderiv(const vco_codec* c, int is_theta, double u)
{
  if (!companded(c, is_theta)) return 1.0;
  if (c->mode == VCO_TANH) {
    double th = tanh(c->gamma * u);
    return c->gamma * (1.0 - th * th) / tanh(c->gamma);
  }
  return 0.5 * PI64 * cos(0.5 * PI64 * u);
}

static double hinv(const vco_codec* c, int is_theta, double hh)
{
  if (!companded(c, is_theta)) return hh;
  if (c->mode == VCO_TANH) return atanh(hh * tanh(c->gamma)) / c->gamma;
  return asin(hh) * (2.0 / PI64);
}

/* n = nint(n_max (1 + h)/2), nint(v) = ceil(floor(2v)/2) = floor(v + 1/2)
 * (round half up, §2.1).  With Q = n_max h / 2:
 *   n_max odd:  n = (n_max+1)/2 + floor(Q)
 *   n_max even: n = n_max/2 + floor(Q + 1/2)
 * which keeps the integer offset out of the floating-point sum (the signed
 * domain of §3). */
static int64_t quantise(uint64_t nmax, double h, double* Qout)
{
  double Q = (double)nmax * h * 0.5;
  int64_t n;
  if (nmax & 1ULL) n = (int64_t)((nmax + 1) / 2) + (int64_t)floor(Q);
  else n = (int64_t)(nmax / 2) + (int64_t)floor(Q + 0.5);
  if (n < 0) n = 0;
  if ((uint64_t)n > nmax) n = (int64_t)nmax;
  if (Qout) *Qout = (nmax & 1ULL) ? Q : Q + 0.5;
  return n;
}

/* ------------------------------------------------------------------------- */
/* encode                                                                     */
/* ------------------------------------------------------------------------- */

static uint64_t mask_bits(int b) { return b >= 64 ? ~0ULL : ((1ULL << b) - 1ULL); }

static uint64_t reserved_code(const vco_codec* c)
{
  /* reading: non-finite input is a precondition violation; it is mapped to
   * the all-ones exponent with every other field zero. */
  return mask_bits(c->e) << (c->m + c->p + c->t);
}

uint64_t vco_encode_detail(const vco_codec* c, float x, float y, float z, vco_detail* d)
{
  vco_detail dd;
  if (!d) d = &dd;
  memset(d, 0, sizeof(*d));
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return reserved_code(c);

  /* reading: signed zeros are canonicalised to +0 before the angles. */
  double X = (double)x + 0.0, Y = (double)y + 0.0, Z = (double)z + 0.0;

  /* ---- magnitude, §2.3 ---- */
  const int prec = c->m + 1;                         /* implicit leading 1 + m stored bits */
  const int64_t Emax_field = (int64_t)mask_bits(c->e) - 1;   /* all-ones exponent reserved */
  const int keep_sub = keeps_subnormals(c);
  const double min_sp = keep_sub ? ldexp(1.0, 1 - c->bias - c->m) : 0.0;
  double rhat;
  int tie = 0;
  if (c->mag_round == VCO_RNE) {
    /* reading: the exact norm is rounded to nearest-even at 1+m bits */
    rhat = vco_round_norm(x, y, z, prec, min_sp, &tie);
  } else {
    /* paper-literal: the single-precision magnitude with the trailing
     * 23-m mantissa bits replaced by zero */
    double r32 = vco_round_norm(x, y, z, 24, 0x1p-149, &tie);
    if (r32 > (double)FLT_MAX) r32 = INFINITY;
    if (r32 != 0.0 && isfinite(r32)) {
      int e32 = ilogb(r32);
      double u = ldexp(1.0, e32 - (prec - 1));
      if (keep_sub && e32 < 1 - c->bias) u = min_sp;
      rhat = floor(r32 / u) * u;
    } else {
      rhat = r32;
    }
  }
  {
    double S = X * X + Y * Y + Z * Z;
    d->r = sqrt(S);
    if (d->r > 0.0 && isfinite(d->r)) {
      int e = ilogb(d->r);
      double u = ldexp(1.0, e - (prec - 1));
      if (min_sp > 0.0 && u < min_sp) u = min_sp;
      double mid = (floor(d->r / u) + 0.5) * u;
      d->mid_rel = fabs(d->r - mid) / d->r;
    }
  }
  if (rhat == 0.0) {
    d->flushed = (d->r > 0.0);
    return 0;
  }
  uint64_t E, M;
  if (!isfinite(rhat)) {
    E = (uint64_t)Emax_field;
    M = mask_bits(c->m);
    d->saturated = 1;
  } else {
    int e = ilogb(rhat);
    int64_t Ei = (int64_t)e + c->bias;
    if (Ei < 1) {
      if (!keep_sub) {
        /* reading: below the smallest normal exponent the vector is stored
         * as the zero code (flush), §2.3 */
        d->flushed = 1;
        return 0;
      }
      E = 0;
      M = (uint64_t)(rhat / min_sp);
    } else if (Ei > Emax_field) {
      /* reading: overflow saturates to the largest finite magnitude */
      E = (uint64_t)Emax_field;
      M = mask_bits(c->m);
      d->saturated = 1;
    } else {
      E = (uint64_t)Ei;
      M = (uint64_t)ldexp(ldexp(rhat, -e) - 1.0, c->m);
    }
  }

  /* ---- angles, §2.1 ---- */
  double theta = atan2(Y, X);            /* reading: two-argument arctangent, theta in [-pi, pi] */
  double rho = hypot(X, Y);
  double phi = atan2(rho, Z);            /* = acos(z/r), evaluated without the ill-conditioned quotient */
  double u_th = theta / PI64;
  double u_ph = 2.0 * (phi / PI64) - 1.0;
  uint64_t nmax_th = vco_nmax_theta(c), nmax_ph = vco_nmax_phi(c);
  double Qt, Qp;
  int64_t n_th = quantise(nmax_th, hmap(c, 1, u_th), &Qt);
  int64_t n_ph = quantise(nmax_ph, hmap(c, 0, u_ph), &Qp);
  d->Q_theta = Qt;
  d->Q_phi = Qp;
  d->n_theta = n_th;
  d->n_phi = n_ph;
  /* window: one single-precision ulp of the angle, in level units */
  d->w_theta = ulp32_of(theta) * fabs(0.5 * (double)nmax_th * hderiv(c, 1, u_th) / PI64);
  d->w_phi = ulp32_of(phi) * fabs(0.5 * (double)nmax_ph * hderiv(c, 0, u_ph) * 2.0 / PI64);

  /* ---- pack, Fig. (comp_regimes): [s][E][M][n_phi][n_theta] ---- */
  uint64_t low;
  if (c->mode == VCO_FRAC) {
    uint64_t T = vco_frac_T(c);
    low = (uint64_t)n_ph * T + (uint64_t)n_th;       /* Eq. (q_split) */
  } else {
    low = ((uint64_t)n_ph << c->t) | (uint64_t)n_th;
  }
  return (E << (c->m + c->p + c->t)) | (M << (c->p + c->t)) | low;
}

uint64_t vco_encode(const vco_codec* c, float x, float y, float z)
{
  return vco_encode_detail(c, x, y, z, NULL);
}

/* ------------------------------------------------------------------------- */
/* decode                                                                     */
/* ------------------------------------------------------------------------- */

/* sin(pi a) and cos(pi a) for a in [-1, 1] with exact argument reduction
 * (a - k/2 is exact), so multiples of 1/2 give exact zeros and ones. */
static void sincospi64(double a, double* s, double* cth)
{
  double k = nearbyint(2.0 * a);
  double f = a - 0.5 * k;
  double sf = sin(PI64 * f), cf = cos(PI64 * f);
  long q = ((long)k % 4 + 4) % 4;
  switch (q) {
    case 0: *s = sf;  *cth = cf;  break;
    case 1: *s = cf;  *cth = -sf; break;
    case 2: *s = -sf; *cth = -cf; break;
    default: *s = -cf; *cth = sf; break;
  }
  if (*s == 0.0) *s = 0.0;
  if (*cth == 0.0) *cth = 0.0;
}

void vco_decode64(const vco_codec* c, uint64_t w, double out[3])
{
  const uint64_t E = (w >> (c->m + c->p + c->t)) & mask_bits(c->e);
  const uint64_t M = (w >> (c->p + c->t)) & mask_bits(c->m);
  const uint64_t low = w & mask_bits(c->p + c->t);
  const double nanv = NAN;
  if (E == mask_bits(c->e)) { out[0] = out[1] = out[2] = nanv; return; }
  double r;
  if (E == 0) {
    if (keeps_subnormals(c) && M != 0) r = (double)M * ldexp(1.0, 1 - c->bias - c->m);
    else { out[0] = out[1] = out[2] = 0.0; return; }
  } else {
    /* r = (1 + M/2^m) 2^(E - b), exactly representable */
    r = ldexp(1.0 + ldexp((double)M, -c->m), (int)E - c->bias);
  }
  uint64_t n_th, n_ph;
  if (c->mode == VCO_FRAC) {
    uint64_t T = vco_frac_T(c);
    if (low >= c->P * T) { out[0] = out[1] = out[2] = nanv; return; }
    n_ph = low / T;
    n_th = low % T;
  } else {
    n_th = low & mask_bits(c->t);
    n_ph = low >> c->t;
  }
  const uint64_t nmax_th = vco_nmax_theta(c), nmax_ph = vco_nmax_phi(c);
  /* half-revolution angles a = angle/pi, Eq. (a_inv) */
  double a_th, a_ph;
  if (!companded(c, 1)) {
    a_th = ((double)(2 * (int64_t)n_th - (int64_t)nmax_th)) / (double)nmax_th;
  } else {
    double hh = ((double)(2 * (int64_t)n_th - (int64_t)nmax_th)) / (double)nmax_th;
    a_th = hinv(c, 1, hh);
  }
  if (!companded(c, 0)) {
    a_ph = (double)n_ph / (double)nmax_ph;
  } else {
    double hh = ((double)(2 * (int64_t)n_ph - (int64_t)nmax_ph)) / (double)nmax_ph;
    a_ph = 0.5 * (hinv(c, 0, hh) + 1.0);
  }
  double st, ct, sp, cp;
  sincospi64(a_th, &st, &ct);
  sincospi64(a_ph, &sp, &cp);
  /* Eq. (cart2sphere) */
  out[0] = r * ct * sp;
  out[1] = r * st * sp;
  out[2] = r * cp;
}

void vco_decode(const vco_codec* c, uint64_t w, float out[3])
{
  double o[3];
  vco_decode64(c, w, o);
  out[0] = (float)o[0];
  out[1] = (float)o[1];
  out[2] = (float)o[2];
}

/* ------------------------------------------------------------------------- */
/* batch forms                                                                */
/* ------------------------------------------------------------------------- */

int vco_max_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int nthr(int n) { return n > 0 ? n : vco_max_threads(); }

void vco_encode_batch(const vco_codec* c, const float* xyz, uint64_t* out, size_t n, int nthreads)
{
  long long N = (long long)n;
#pragma omp parallel for schedule(static) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) out[i] = vco_encode(c, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
}

void vco_encode_detail_batch(const vco_codec* c, const float* xyz, uint64_t* out, double* q5,
                             int32_t* flags, size_t n, int nthreads)
{
  long long N = (long long)n;
#pragma omp parallel for schedule(static) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) {
    vco_detail d;
    out[i] = vco_encode_detail(c, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], &d);
    if (q5) {
      q5[5 * i + 0] = d.Q_theta;
      q5[5 * i + 1] = d.w_theta;
      q5[5 * i + 2] = d.Q_phi;
      q5[5 * i + 3] = d.w_phi;
      q5[5 * i + 4] = d.mid_rel;
    }
    if (flags) flags[i] = (d.saturated ? 1 : 0) | (d.flushed ? 2 : 0);
  }
}

void vco_decode_batch(const vco_codec* c, const uint64_t* w, float* xyz, size_t n, int nthreads)
{
  long long N = (long long)n;
#pragma omp parallel for schedule(static) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) vco_decode(c, w[i], xyz + 3 * i);
}

void vco_decode64_batch(const vco_codec* c, const uint64_t* w, double* xyz, size_t n, int nthreads)
{
  long long N = (long long)n;
#pragma omp parallel for schedule(static) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) vco_decode64(c, w[i], xyz + 3 * i);
}

/* c = alpha a + b on compressed operands (§5): decode both, one single-precision
 * fused multiply-add per component, encode the result. */
void vco_axpy_batch(const vco_codec* c, float alpha, const uint64_t* a, const uint64_t* b,
                    uint64_t* out, float* c32, double* c64, size_t n, int nthreads)
{
  long long N = (long long)n;
#pragma omp parallel for schedule(static) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) {
    float A[3], B[3], C[3];
    vco_decode(c, a[i], A);
    vco_decode(c, b[i], B);
    for (int k = 0; k < 3; k++) C[k] = vco_rn32_fma(alpha, A[k], B[k]);
    if (out) out[i] = vco_encode(c, C[0], C[1], C[2]);
    if (c32) for (int k = 0; k < 3; k++) c32[3 * i + k] = C[k];
    if (c64) {
      double A64[3], B64[3];
      vco_decode64(c, a[i], A64);
      vco_decode64(c, b[i], B64);
      for (int k = 0; k < 3; k++) c64[3 * i + k] = (double)alpha * A64[k] + B64[k];
    }
  }
}

double vco_dot(const vco_codec* c, const uint64_t* a, const uint64_t* b, size_t n, int nthreads)
{
  long long N = (long long)n;
  long double total = 0.0L;
#pragma omp parallel for schedule(static) reduction(+ : total) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) {
    double A[3], B[3];
    vco_decode64(c, a[i], A);
    vco_decode64(c, b[i], B);
    total += (long double)A[0] * B[0] + (long double)A[1] * B[1] + (long double)A[2] * B[2];
  }
  return (double)total;
}

double vco_norm2(const vco_codec* c, const uint64_t* a, size_t n, int nthreads)
{
  long long N = (long long)n;
  long double total = 0.0L;
#pragma omp parallel for schedule(static) reduction(+ : total) num_threads(nthr(nthreads))
  for (long long i = 0; i < N; i++) {
    double A[3];
    vco_decode64(c, a[i], A);
    total += (long double)A[0] * A[0] + (long double)A[1] * A[1] + (long double)A[2] * A[2];
  }
  return (double)total;
}

void vco_apply(const vco_codec* c, const float* M, int rows, int cols, const uint64_t* U,
               double* out, size_t n_elem, int nthreads)
{
  long long N = (long long)n_elem;
#pragma omp parallel for schedule(static) num_threads(nthr(nthreads))
  for (long long e = 0; e < N; e++) {
    double X[3];
    double* o = out + (size_t)e * rows * 3;
    for (int i = 0; i < rows * 3; i++) o[i] = 0.0;
    for (int j = 0; j < cols; j++) {
      vco_decode64(c, U[(size_t)e * cols + j], X);
      for (int i = 0; i < rows; i++) {
        double mij = (double)M[(size_t)i * cols + j];
        o[3 * i + 0] += mij * X[0];
        o[3 * i + 1] += mij * X[1];
        o[3 * i + 2] += mij * X[2];
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* error statistics of the codec (the error measures of §2.2-§2.3)            */
/* ------------------------------------------------------------------------- */

/* magnitude r_hat of a regular code from its fields (§2.3); 0 for the zero code,
 * -1 for the reserved code */
static double code_magnitude(const vco_codec* c, uint64_t w)
{
  const uint64_t E = (w >> (c->m + c->p + c->t)) & mask_bits(c->e);
  const uint64_t M = (w >> (c->p + c->t)) & mask_bits(c->m);
  if (E == mask_bits(c->e)) return -1.0;
  if (E == 0) return keeps_subnormals(c) ? (double)M * ldexp(1.0, 1 - c->bias - c->m) : 0.0;
  return ldexp(1.0 + ldexp((double)M, -c->m), (int)E - c->bias);
}

static int bin_of(double e, const double* edges, int nedges)
{
  int k = 0;
  while (k < nedges && edges[k] <= e) k++;
  return k;
}

void vco_error_hist(const vco_codec* c, const float* xyz, size_t n, const double* edges, int nedges,
                    uint64_t* counts, double* stats, int nthreads)
{
  const int nb = nedges + 1;
  const int T = nthr(nthreads);
  uint64_t* loc = (uint64_t*)calloc((size_t)T * (3 * nb + 1), sizeof(uint64_t));
  double* ls = (double*)calloc((size_t)T * 9, sizeof(double));
  long long N = (long long)n;
#pragma omp parallel num_threads(T)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    uint64_t* h = loc + (size_t)tid * (3 * nb + 1);
    double* s = ls + (size_t)tid * 9;
#pragma omp for schedule(static)
    for (long long i = 0; i < N; i++) {
      const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
      if (!isfinite(x) || !isfinite(y) || !isfinite(z) || (x == 0.0f && y == 0.0f && z == 0.0f)) {
        h[3 * nb]++;
        continue;
      }
      vco_detail d;
      const uint64_t w = vco_encode_detail(c, x, y, z, &d);
      const double rh = code_magnitude(c, w);
      if (d.saturated || d.flushed || rh <= 0.0) {
        h[3 * nb]++;
        continue;
      }
      double xh[3];
      vco_decode64(c, w, xh);
      const double X = x, Y = y, Z = z;
      const double r = sqrt(X * X + Y * Y + Z * Z);
      const double dx = xh[0] - X, dy = xh[1] - Y, dz = xh[2] - Z;
      const double cx = Y * xh[2] - Z * xh[1], cy = Z * xh[0] - X * xh[2], cz = X * xh[1] - Y * xh[0];
      double e[3];
      e[0] = sqrt(dx * dx + dy * dy + dz * dz) / r;                                   /* |x_hat - x| / |x| */
      e[1] = atan2(sqrt(cx * cx + cy * cy + cz * cz), X * xh[0] + Y * xh[1] + Z * xh[2]); /* angle */
      e[2] = fabs(rh - r) / r;                                                        /* |r_hat - r| / r */
      for (int k = 0; k < 3; k++) {
        h[k * nb + bin_of(e[k], edges, nedges)]++;
        s[3 * k] += e[k];
        s[3 * k + 1] += e[k] * e[k];
        if (e[k] > s[3 * k + 2]) s[3 * k + 2] = e[k];
      }
    }
  }
  for (int j = 0; j < 3 * nb + 1; j++) counts[j] = 0;
  for (int k = 0; k < 9; k++) stats[k] = 0.0;
  for (int t = 0; t < T; t++) {
    for (int j = 0; j < 3 * nb + 1; j++) counts[j] += loc[(size_t)t * (3 * nb + 1) + j];
    for (int k = 0; k < 3; k++) {
      stats[3 * k] += ls[t * 9 + 3 * k];
      stats[3 * k + 1] += ls[t * 9 + 3 * k + 1];
      if (ls[t * 9 + 3 * k + 2] > stats[3 * k + 2]) stats[3 * k + 2] = ls[t * 9 + 3 * k + 2];
    }
  }
  free(loc);
  free(ls);
}

/* ------------------------------------------------------------------------- */
/* divergence of a compressed flux (§4, Alg. fr_fdiv_comp)                    */
/* ------------------------------------------------------------------------- */

/* For every element i and solution point j the flux codes F[i][j][0..np) are decompressed to
 * X (np rows of 3); every solution point k then receives d . X_p with
 * d = (D[j][k], D[ns + j][k], D[2 ns + j][k]), D the 3 ns x ns divergence operator.  FP64
 * accumulation in the algorithm's loop order. */
void vco_flux_div(const vco_codec* c, const float* D, int ns, int np, const uint64_t* F, double* out,
                  size_t n_elem, int nthreads)
{
  long long N = (long long)n_elem;
#pragma omp parallel num_threads(nthr(nthreads))
  {
    double* X = (double*)malloc(sizeof(double) * 3 * (size_t)np);
#pragma omp for schedule(static)
    for (long long i = 0; i < N; i++) {
      double* o = out + (size_t)i * ns * np;
      for (int t = 0; t < ns * np; t++) o[t] = 0.0;
      for (int j = 0; j < ns; j++) {
        for (int p = 0; p < np; p++) vco_decode64(c, F[((size_t)i * ns + j) * np + p], X + 3 * p);
        for (int k = 0; k < ns; k++) {
          const double d0 = D[(size_t)j * ns + k];
          const double d1 = D[(size_t)(ns + j) * ns + k];
          const double d2 = D[(size_t)(2 * ns + j) * ns + k];
          for (int p = 0; p < np; p++) o[(size_t)k * np + p] += d0 * X[3 * p] + d1 * X[3 * p + 1] + d2 * X[3 * p + 2];
        }
      }
    }
    free(X);
  }
}
