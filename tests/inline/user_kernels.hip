// A kernel written against the public inline header only (test infrastructure): it encodes a
// vector, stores the code, decodes the code again and forms the dot product of consecutive
// codes, all inside one user kernel.  The tests compare it with the library's entry points.
#include <string.h>

#include <hip/hip_runtime.h>

#include "../../include/vc_ext.h"
#include "../../include/vc_inline.hpp"

__global__ void k_user_roundtrip(const float* __restrict__ xyz, uint64_t* __restrict__ codes,
                                 float* __restrict__ back, float* __restrict__ dots, size_t n, vc_inline::Params P)
{
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t w = vc_inline::encode(P, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
  codes[i] = w;
  vc_inline::decode(P, w, back[3 * i], back[3 * i + 1], back[3 * i + 2]);
  const size_t j = i + 1 < n ? i + 1 : i;
  const uint64_t wj = vc_inline::encode(P, xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2]);
  dots[i] = vc_inline::dot(P, w, wj);
}

extern "C" int user_roundtrip(const vc_codec* c, const float* xyz, uint64_t* codes, float* back, float* dots,
                              size_t n, hipStream_t stream)
{
  vc_inline::Params P;
  const int st = vcx_inline_params(c, &P, sizeof P);
  if (st != VC_SUCCESS) return st;
  if (n == 0) return 0;
  const unsigned grid = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_user_roundtrip, dim3(grid), dim3(256), 0, stream, xyz, codes, back, dots, n, P);
  return hipGetLastError() == hipSuccess ? 0 : VC_ERROR_LAUNCH;
}
