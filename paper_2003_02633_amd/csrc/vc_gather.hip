// vc_gather.hip -- indexed (random-access) decode and encode of compressed 3-vectors.
//
// Fixed-rate codes can be addressed individually, the property the paper asks of an inline
// compression for unstructured data (§1): an interface kernel of flux reconstruction reads the
// flux-point values of two neighbouring elements through a connectivity array (Table fr_nse,
// steps 2 and 8).  Here
//   gather : out[i] = decode(codes[idx[i]])           (idx read coalesced, codes at random)
//   scatter: codes[idx[i]] = encode(xyz[i])           (the inverse, for a permutation)
// Indices at or beyond the source/destination length are not dereferenced: the gather writes
// NaN for them and the scatter skips them.  The uncompressed twin gathers float32 AoS vectors.
#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

constexpr int GS_BS = 256;

template <class L, int MODE>
__global__ __launch_bounds__(GS_BS) void k_gather_decode(const uint64_t* __restrict__ codes, size_t n_src,
                                                         const uint32_t* __restrict__ idx, size_t n,
                                                         float* __restrict__ out, Params P)
{
  for (size_t i = (size_t)blockIdx.x * GS_BS + threadIdx.x; i < n; i += (size_t)gridDim.x * GS_BS) {
    const uint32_t j = __builtin_nontemporal_load(idx + i);
    float x, y, z;
    if (j < n_src) {
      decode_vec<L, MODE>(codes[j], P, x, y, z);
    } else {
      x = y = z = __builtin_nanf("");
    }
    out[3 * i] = x; out[3 * i + 1] = y; out[3 * i + 2] = z;
  }
}

template <class L, int MODE, int PREC>
__global__ __launch_bounds__(GS_BS) void k_scatter_encode(const float* __restrict__ xyz, const uint32_t* __restrict__ idx,
                                                          size_t n, uint64_t* __restrict__ codes, size_t n_dst,
                                                          Params P)
{
  for (size_t i = (size_t)blockIdx.x * GS_BS + threadIdx.x; i < n; i += (size_t)gridDim.x * GS_BS) {
    const uint32_t j = __builtin_nontemporal_load(idx + i);
    if (j < n_dst) codes[j] = encode_vec<L, MODE, PREC>(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], P);
  }
}

__global__ __launch_bounds__(GS_BS) void k_gather_f32(const float* __restrict__ src, size_t n_src,
                                                      const uint32_t* __restrict__ idx, size_t n,
                                                      float* __restrict__ out)
{
  for (size_t i = (size_t)blockIdx.x * GS_BS + threadIdx.x; i < n; i += (size_t)gridDim.x * GS_BS) {
    const uint32_t j = __builtin_nontemporal_load(idx + i);
    float x, y, z;
    if (j < n_src) {
      x = src[3 * (size_t)j]; y = src[3 * (size_t)j + 1]; z = src[3 * (size_t)j + 2];
    } else {
      x = y = z = __builtin_nanf("");
    }
    out[3 * i] = x; out[3 * i + 1] = y; out[3 * i + 2] = z;
  }
}

static inline unsigned gs_grid(size_t n)
{
  size_t g = (n + GS_BS - 1) / GS_BS;
  if (g > (1u << 30)) g = 1u << 30;
  return (unsigned)(g < 1 ? 1 : g);
}

template <class L, int MODE, int PREC>
static vc_status gather_t(const Resolved& R, const uint64_t* codes, size_t n_src, const uint32_t* idx, size_t n,
                          float* out, hipStream_t s)
{
  hipLaunchKernelGGL((k_gather_decode<L, MODE>), dim3(gs_grid(n)), dim3(GS_BS), 0, s, codes, n_src, idx, n, out, R.P);
  return launch_status();
}

template <class L, int MODE, int PREC>
static vc_status scatter_t(const Resolved& R, const float* xyz, const uint32_t* idx, size_t n, uint64_t* codes,
                           size_t n_dst, hipStream_t s)
{
  hipLaunchKernelGGL((k_scatter_encode<L, MODE, PREC>), dim3(gs_grid(n)), dim3(GS_BS), 0, s, xyz, idx, n, codes,
                     n_dst, R.P);
  return launch_status();
}

static bool overlap(const void* p, size_t pb, const void* q, size_t qb)
{
  const uintptr_t a0 = (uintptr_t)p, b0 = (uintptr_t)q;
  return a0 < b0 + qb && b0 < a0 + pb;
}

}  // namespace vc

using namespace vc;

extern "C" vc_status vc_gather_decode(const vc_codec* c, const uint64_t* codes, size_t n_src, const uint32_t* idx,
                                      size_t n, float* out, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (n == 0) return VC_SUCCESS;
  if ((!codes && n_src) || !idx || !out) return VC_ERROR_INVALID_VALUE;
  if (((uintptr_t)codes & 7u) || ((uintptr_t)idx & 3u) || ((uintptr_t)out & 3u)) return VC_ERROR_MISALIGNED;
  if (overlap(out, 12 * n, codes, 8 * n_src) || overlap(out, 12 * n, idx, 4 * n)) return VC_ERROR_OVERLAP;
  VC_DISPATCH_NOPREC(R, gather_t, R, codes, n_src, idx, n, out, stream);
}

extern "C" vc_status vc_scatter_encode(const vc_codec* c, const float* xyz, const uint32_t* idx, size_t n,
                                       uint64_t* codes, size_t n_dst, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (n == 0) return VC_SUCCESS;
  if (!xyz || !idx || (!codes && n_dst)) return VC_ERROR_INVALID_VALUE;
  if (((uintptr_t)codes & 7u) || ((uintptr_t)idx & 3u) || ((uintptr_t)xyz & 3u)) return VC_ERROR_MISALIGNED;
  if (overlap(codes, 8 * n_dst, xyz, 12 * n) || overlap(codes, 8 * n_dst, idx, 4 * n)) return VC_ERROR_OVERLAP;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;
  VC_DISPATCH(R, scatter_t, R, xyz, idx, n, codes, n_dst, stream);
}

extern "C" vc_status vcb_gather_f32(const float* src, size_t n_src, const uint32_t* idx, size_t n, float* out,
                                    hipStream_t stream)
{
  if (n == 0) return VC_SUCCESS;
  if ((!src && n_src) || !idx || !out) return VC_ERROR_INVALID_VALUE;
  if (((uintptr_t)src & 3u) || ((uintptr_t)idx & 3u) || ((uintptr_t)out & 3u)) return VC_ERROR_MISALIGNED;
  if (overlap(out, 12 * n, src, 12 * n_src) || overlap(out, 12 * n, idx, 4 * n)) return VC_ERROR_OVERLAP;
  hipLaunchKernelGGL(k_gather_f32, dim3(gs_grid(n)), dim3(GS_BS), 0, stream, src, n_src, idx, n, out);
  return launch_status();
}
