/*
 * vco.h -- CPU oracle for the inline 3-vector compression of Trojak & Witherden,
 * "Inline Vector Compression for Computational Physics" (arXiv 2003.02633).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links, loads or calls it, and the two share no code.
 *
 * Arithmetic: FP64 and integers.  Where the paper's definition is an exact
 * real-number statement (round-to-nearest of a real magnitude, floor of a real
 * level coordinate), the oracle decides it exactly (expansion arithmetic for
 * signs of sums of squares, exactly-rounded single-precision sums).
 *
 * Parity status of each entry point is listed in oracle/README.md.
 */
#ifndef VCO_H
#define VCO_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VCO_PLAIN = 0, VCO_TANH = 1, VCO_COS = 2, VCO_FRAC = 3 };
enum { VCO_RNE = 0, VCO_TRUNC = 1 };
enum { VCO_COMP_PHI = 1, VCO_COMP_THETA = 2 };

/* Codec parameters, paper notation <s,e,m>-p-t (§2.3) plus the variant knobs of
 * §2.4 (fractional split) and §2.5 (companding). */
typedef struct {
  int s, e, m, p, t;   /* sign bits, exponent bits, mantissa bits, n_phi bits, n_theta bits */
  int bias;            /* exponent bias b_e (b_7 = 80, b_8 = 127), §2.3 */
  int mode;            /* VCO_PLAIN / VCO_TANH / VCO_COS / VCO_FRAC */
  int mag_round;       /* VCO_RNE (default) or VCO_TRUNC (paper-literal mantissa truncation) */
  int compand_mask;    /* which angles a companding map applies to */
  double gamma;        /* tanh companding parameter, §2.5 */
  uint64_t P;          /* fractional split: n_phi_max + 1, §2.4 */
} vco_codec;

/* Per-vector detail of an encode, for the window rule used in GPU parity. */
typedef struct {
  double Q_theta, w_theta;  /* exact pre-floor level coordinate and 1-ulp window (level units) */
  double Q_phi, w_phi;
  int64_t n_theta, n_phi;   /* chosen levels */
  double r;                 /* FP64 estimate of the exact magnitude */
  double mid_rel;           /* |r - nearest rounding midpoint| / r for the magnitude field */
  int saturated;            /* 1 when the magnitude was clamped to the largest code */
  int flushed;              /* 1 when the magnitude underflowed to the zero code */
} vco_detail;

int      vco_check(const vco_codec* c);                   /* 0 if the parameters are valid */
uint64_t vco_nmax_theta(const vco_codec* c);
uint64_t vco_nmax_phi(const vco_codec* c);
uint64_t vco_frac_T(const vco_codec* c);

uint64_t vco_encode(const vco_codec* c, float x, float y, float z);
uint64_t vco_encode_detail(const vco_codec* c, float x, float y, float z, vco_detail* d);
void     vco_decode64(const vco_codec* c, uint64_t w, double out[3]);
void     vco_decode(const vco_codec* c, uint64_t w, float out[3]);

/* exact single-precision result of alpha*a + b (one rounding) */
float    vco_rn32_fma(float alpha, float a, float b);
/* exact magnitude rounded to `prec` significant bits (RNE); flags exact ties */
double   vco_round_norm(float x, float y, float z, int prec, double min_spacing, int* tie);
/* sign of the exact sum v[0]+...+v[n-1] of finite doubles */
int      vco_exact_sign(const double* v, int n);

/* batch forms (OpenMP over vectors); nthreads <= 0 uses the OpenMP default */
void vco_encode_batch(const vco_codec* c, const float* xyz, uint64_t* out, size_t n, int nthreads);
/* q5[i] = {Q_theta, w_theta, Q_phi, w_phi, mid_rel}; flags bit0 saturated, bit1 flushed */
void vco_encode_detail_batch(const vco_codec* c, const float* xyz, uint64_t* out, double* q5,
                             int32_t* flags, size_t n, int nthreads);
void vco_decode_batch(const vco_codec* c, const uint64_t* w, float* xyz, size_t n, int nthreads);
void vco_decode64_batch(const vco_codec* c, const uint64_t* w, double* xyz, size_t n, int nthreads);
void vco_axpy_batch(const vco_codec* c, float alpha, const uint64_t* a, const uint64_t* b,
                    uint64_t* out, float* c32, double* c64, size_t n, int nthreads);
double vco_dot(const vco_codec* c, const uint64_t* a, const uint64_t* b, size_t n, int nthreads);
double vco_norm2(const vco_codec* c, const uint64_t* a, size_t n, int nthreads);
/* out[e][i][k] = sum_j M[i][j] * decode(U[e][j])[k], FP64 */
void vco_apply(const vco_codec* c, const float* M, int rows, int cols, const uint64_t* U,
               double* out, size_t n_elem, int nthreads);
int vco_max_threads(void);

/* Error statistics of encode -> FP64 decode over a batch of vectors (the error measures of
 * §2.2-§2.3), for each finite non-zero input whose code is neither flushed nor saturated:
 *   k = 0: |x_hat - x| / |x|,  k = 1: the angle between x and x_hat,  k = 2: |r_hat - |x|| / |x|
 * (x_hat the FP64 decode, r_hat the code's magnitude).  Histogram bin = number of edges <= e
 * (edges ascending, 0..nedges): counts[k (nedges+1) + bin]; counts[3 (nedges+1)] = vectors left
 * out.  stats[3k] = sum e, stats[3k+1] = sum e^2, stats[3k+2] = max e. */
/* Divergence of a compressed flux, Alg. (fr_fdiv_comp): out[i][k][p] = sum_j sum_c
 * D[c ns + j][k] decode(F[i][j][p])[c], D float32 [3 ns][ns] row-major, F codes [n_elem][ns][np],
 * out FP64 [n_elem][ns][np]. */
void vco_flux_div(const vco_codec* c, const float* D, int ns, int np, const uint64_t* F, double* out,
                  size_t n_elem, int nthreads);

void vco_error_hist(const vco_codec* c, const float* xyz, size_t n, const double* edges, int nedges,
                    uint64_t* counts, double* stats, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
