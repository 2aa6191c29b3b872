// Runs the host build of the device codec (tests/hostemu/vc_hostemu.cpp: vc_device.hpp and the
// codec resolution of vc_params.hpp compiled for the CPU) over edge-case and random inputs for
// every codec the library accepts, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure, CPU only).  The exact magnitude path is driven
// directly as well, at every precision and subnormal setting it is used with.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/vc.h"

extern "C" {
int emu_encode(const vc_codec* c, const float* xyz, uint64_t* out, size_t n);
int emu_decode(const vc_codec* c, const uint64_t* w, float* out, size_t n);
int emu_dot_pair(const vc_codec* c, const uint64_t* a, const uint64_t* b, float* out, size_t n);
int emu_exact_norm(float x, float y, float z, int prec, int keep_sub, uint32_t* j, int* g);
int emu_magnitude_checked(const vc_codec* c, const uint64_t* w, float* out, size_t n);
}

static uint64_t state = 0x2545f4914f6cdd1dull;
static uint64_t next64()                          // splitmix64
{
  uint64_t z = (state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static float bits_float(uint32_t u)
{
  float f;
  memcpy(&f, &u, 4);
  return f;
}

int main()
{
  const size_t n = 4096;
  std::vector<float> xyz(3 * n), out(3 * n), d(n);
  std::vector<uint64_t> w(n), r(n);
  const float edge[] = {0.0f, -0.0f, 1.0f, -1.0f, 1e-30f, 1e30f, 1e-45f, 1.17549435e-38f, 3.4028235e38f,
                        -3.4028235e38f, INFINITY, -INFINITY, NAN, 0.5f, 2.0f, 16777215.0f, 8192.0f};
  const size_t ne = sizeof edge / sizeof edge[0];
  size_t i = 0;
  for (size_t a = 0; a < ne; a++)
    for (size_t b = 0; b < ne; b++)
      for (size_t c = 0; c < ne && i < n; c += 2, i++) {
        xyz[3 * i] = edge[a]; xyz[3 * i + 1] = edge[b]; xyz[3 * i + 2] = edge[c];
      }
  for (; i < n; i++)
    for (int k = 0; k < 3; k++) {
      const uint64_t u = next64();
      // half arbitrary bit patterns, half finite values spread over the float32 exponent range
      xyz[3 * i + k] = (i & 1) ? bits_float((uint32_t)u)
                               : bits_float(((uint32_t)u & 0x807fffffu) | ((uint32_t)((u >> 32) % 254 + 1) << 23));
    }
  for (size_t k = 0; k < n; k++) r[k] = next64();
  r[0] = 0; r[1] = ~0ull;

  int runs = 0;
  for (uint32_t layout = 0; layout < 4; layout++)
    for (uint32_t mode = 0; mode < 4; mode++)
      for (uint32_t mag = 0; mag < 2; mag++)
        for (uint32_t prec = 0; prec < 2; prec++) {
          vc_codec c;
          memset(&c, 0, sizeof c);
          c.struct_size = sizeof(vc_codec);
          c.layout = layout; c.mode = mode; c.mag_round = mag; c.precision = prec;
          c.compand_mask = VC_COMPAND_PHI | VC_COMPAND_THETA;
          c.gamma = 0.5f;
          // the fractional split at a moderate and at the largest accepted level count
          for (uint64_t P : {163840ull, 1ull << 24}) {
            c.frac_P = P;
            if (emu_encode(&c, xyz.data(), w.data(), n) != 0) break;   // combination not built
            if (emu_decode(&c, w.data(), out.data(), n) != 0) return 2;
            if (emu_decode(&c, r.data(), out.data(), n) != 0) return 2;
            if (emu_dot_pair(&c, w.data(), r.data(), d.data(), n) != 0) return 2;
            if (emu_magnitude_checked(&c, r.data(), d.data(), n) != 0) return 2;
            runs++;
            if (mode != VC_MODE_FRACSPLIT) break;
          }
        }
  for (size_t k = 0; k < n; k++) {
    const float x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) continue;
    uint32_t j;
    int g;
    emu_exact_norm(x, y, z, 23, 0, &j, &g);
    emu_exact_norm(x, y, z, 24, 0, &j, &g);
    emu_exact_norm(x, y, z, 24, 1, &j, &g);
  }
  printf("codecs run: %d\n", runs);
  return runs > 0 ? 0 : 1;
}
