/* Runs every entry point of the CPU oracle over edge-case and random inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure, CPU only).  Exits 0 when
 * every call returned; the sanitizers abort with a report on an out-of-bounds access, an
 * overflow of a signed integer, a bad shift or a misaligned access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/vco.h"

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint64_t next64(void)                      /* splitmix64 */
{
  uint64_t z = (state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static float rnd_float(void)                      /* any bit pattern: normals, subnormals, inf, nan */
{
  uint32_t u = (uint32_t)next64();
  float f;
  memcpy(&f, &u, 4);
  return f;
}

#define NV 2048
static float xyz[3 * NV];
static uint64_t w1[NV], w2[NV], w3[NV];
static float f3[3 * NV], c32[3 * NV];
static double d3[3 * NV], c64[3 * NV], q5[5 * NV];
static int32_t flags[NV];

static void fill_inputs(void)
{
  const float edge[] = {0.0f, -0.0f, 1.0f, -1.0f, 1e-30f, 1e30f, 1e-45f, 1.17549435e-38f,
                        3.4028235e38f, -3.4028235e38f, INFINITY, -INFINITY, NAN, 0.5f, 2.0f};
  const int ne = (int)(sizeof edge / sizeof edge[0]);
  int i = 0;
  for (int a = 0; a < ne && i < NV; a++)
    for (int b = 0; b < ne && i < NV; b += 2)
      for (int d = 0; d < ne && i < NV; d += 3, i++) {
        xyz[3 * i] = edge[a]; xyz[3 * i + 1] = edge[b]; xyz[3 * i + 2] = edge[d];
      }
  for (; i < NV; i++)
    for (int k = 0; k < 3; k++) xyz[3 * i + k] = (i & 1) ? rnd_float() : (float)((int64_t)next64() % 2001 - 1000) / 7.0f;
}

static void run_codec(const vco_codec* c)
{
  if (vco_check(c) != 0) { fprintf(stderr, "invalid codec\n"); exit(2); }
  vco_encode_batch(c, xyz, w1, NV, 1);
  vco_encode_detail_batch(c, xyz, w2, q5, flags, NV, 1);
  for (int i = 0; i < NV; i++) w3[i] = next64();           /* arbitrary codes, reserved included */
  w3[0] = 0; w3[1] = ~0ull;
  vco_decode_batch(c, w1, f3, NV, 1);
  vco_decode_batch(c, w3, f3, NV, 1);
  vco_decode64_batch(c, w3, d3, NV, 1);
  vco_axpy_batch(c, 0.7f, w1, w3, w2, c32, c64, NV, 1);
  volatile double s = vco_dot(c, w1, w3, NV, 1) + vco_norm2(c, w3, NV, 1);
  (void)s;
  float M[6 * 5];
  for (int i = 0; i < 30; i++) M[i] = (float)i / 7.0f - 2.0f;
  vco_apply(c, M, 6, 5, w3, d3, 300, 1);             /* 300 x 5 codes in, 300 x 6 x 3 out */
  /* flux divergence: q = 2 points a direction, ns = 8, np = 5, D [3 ns][ns] */
  float D[3 * 8 * 8];
  for (int i = 0; i < 3 * 8 * 8; i++) D[i] = (float)(i % 7) - 3.0f;
  vco_flux_div(c, D, 8, 5, w3, d3, NV / 40, 1);       /* 51 x 8 x 5 codes and outputs */
  double edges[11];
  for (int i = 0; i < 11; i++) edges[i] = pow(10.0, -12.0 + i);
  uint64_t counts[3 * 12 + 1];
  double stats[9];
  vco_error_hist(c, xyz, NV, edges, 11, counts, stats, 1);
  int tie;
  for (int i = 0; i < 64; i++) {
    float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (isfinite(x) && isfinite(y) && isfinite(z)) (void)vco_round_norm(x, y, z, 23, 0.0, &tie);
  }
}

int main(void)
{
  fill_inputs();
  const int L[4][6] = {{0, 7, 22, 17, 18, 80}, {0, 7, 23, 17, 17, 80}, {0, 8, 23, 16, 17, 127}, {1, 8, 23, 16, 16, 127}};
  int n = 0;
  for (int l = 0; l < 4; l++)
    for (int mode = 0; mode < 4; mode++)
      for (int mr = 0; mr < 2; mr++) {
        vco_codec c = {L[l][0], L[l][1], L[l][2], L[l][3], L[l][4], L[l][5], mode, mr, 3, 0.5,
                       mode == VCO_FRAC ? 163840ull : 0ull};
        if (mode == VCO_FRAC && l == 3) c.P = 1ull << 15;
        if (vco_check(&c) != 0) continue;
        run_codec(&c);
        n++;
      }
  printf("codecs run: %d\n", n);
  return n > 0 ? 0 : 1;
}
