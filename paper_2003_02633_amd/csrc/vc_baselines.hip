// vc_baselines.hip -- uncompressed streaming kernels used as measurement references:
// float32 axpy (12 B per 3-vector), bf16/fp16 axpy padded to 8 B per 3-vector, copy.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_axpy_f32(float alpha, const float* __restrict__ a,
                                                  const float* __restrict__ b, float* __restrict__ c, size_t n4,
                                                  size_t n)
{
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
    const f32x4 va = __builtin_nontemporal_load((const f32x4*)a + i);
    const f32x4 vb = __builtin_nontemporal_load((const f32x4*)b + i);
    f32x4 vc;
    vc[0] = __builtin_fmaf(alpha, va[0], vb[0]);
    vc[1] = __builtin_fmaf(alpha, va[1], vb[1]);
    vc[2] = __builtin_fmaf(alpha, va[2], vb[2]);
    vc[3] = __builtin_fmaf(alpha, va[3], vb[3]);
    __builtin_nontemporal_store(vc, (f32x4*)c + i);
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    c[i] = __builtin_fmaf(alpha, a[i], b[i]);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f32_to_bf16(float f)
{
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;         // NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;                // nearest-even
}
__device__ __forceinline__ float f16_to_f32(uint32_t h) { return __half2float(__ushort_as_half((unsigned short)h)); }
__device__ __forceinline__ uint32_t f32_to_f16(float f) { return __half_as_ushort(__float2half_rn(f)); }

// one 3-vector (4 x 16 bit) per 8 bytes; two vectors per lane and step (16-byte accesses)
template <bool BF16>
__global__ __launch_bounds__(256) void k_axpy_h4(float alpha, const uint16_t* __restrict__ a,
                                                 const uint16_t* __restrict__ b, uint16_t* __restrict__ c,
                                                 size_t npairs, size_t nvec)
{
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < npairs; i += stride) {
    const u32x4 va = __builtin_nontemporal_load((const u32x4*)a + i);
    const u32x4 vb = __builtin_nontemporal_load((const u32x4*)b + i);
    u32x4 vc;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t lo_a = va[k] & 0xffffu, hi_a = va[k] >> 16, lo_b = vb[k] & 0xffffu, hi_b = vb[k] >> 16;
      float x0, x1;
      if (BF16) {
        x0 = __builtin_fmaf(alpha, bf16_to_f32(lo_a), bf16_to_f32(lo_b));
        x1 = __builtin_fmaf(alpha, bf16_to_f32(hi_a), bf16_to_f32(hi_b));
        vc[k] = f32_to_bf16(x0) | (f32_to_bf16(x1) << 16);
      } else {
        x0 = __builtin_fmaf(alpha, f16_to_f32(lo_a), f16_to_f32(lo_b));
        x1 = __builtin_fmaf(alpha, f16_to_f32(hi_a), f16_to_f32(hi_b));
        vc[k] = f32_to_f16(x0) | (f32_to_f16(x1) << 16);
      }
    }
    // the padding lane (4th value of each vector) stays zero
    vc[1] &= 0x0000ffffu;
    vc[3] &= 0x0000ffffu;
    __builtin_nontemporal_store(vc, (u32x4*)c + i);
  }
  if ((nvec & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t v = nvec - 1;
    for (int k = 0; k < 3; k++) {
      const uint32_t ha = a[4 * v + k], hb = b[4 * v + k];
      if (BF16) c[4 * v + k] = (uint16_t)f32_to_bf16(__builtin_fmaf(alpha, bf16_to_f32(ha), bf16_to_f32(hb)));
      else c[4 * v + k] = (uint16_t)f32_to_f16(__builtin_fmaf(alpha, f16_to_f32(ha), f16_to_f32(hb)));
    }
    c[4 * v + 3] = 0;
  }
}

__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ s, u32x4* __restrict__ d, size_t n16)
{
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}

static unsigned grid_of(size_t items)
{
  size_t g = (items + 255) / 256;
  if (g < 1) g = 1;
  if (g > (1u << 30)) g = 1u << 30;
  return (unsigned)g;
}

}  // namespace vc

using namespace vc;

extern "C" {

vc_status vcb_axpy_f32(float alpha, const float* a, const float* b, float* c, size_t nfloats, hipStream_t stream)
{
  if (nfloats == 0) return VC_SUCCESS;
  if (!a || !b || !c) return VC_ERROR_INVALID_VALUE;
  if ((((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15u) != 0) return VC_ERROR_MISALIGNED;
  const size_t n4 = nfloats / 4;
  hipLaunchKernelGGL(k_axpy_f32, dim3(grid_of(n4 ? n4 : 1)), dim3(256), 0, stream, alpha, a, b, c, n4, nfloats);
  return launch_status();
}

static vc_status axpy_h4(bool bf16, float alpha, const uint16_t* a, const uint16_t* b, uint16_t* c, size_t nvec,
                         hipStream_t stream)
{
  if (nvec == 0) return VC_SUCCESS;
  if (!a || !b || !c) return VC_ERROR_INVALID_VALUE;
  if ((((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15u) != 0) return VC_ERROR_MISALIGNED;
  const size_t np = nvec / 2;
  if (bf16)
    hipLaunchKernelGGL(k_axpy_h4<true>, dim3(grid_of(np ? np : 1)), dim3(256), 0, stream, alpha, a, b, c, np, nvec);
  else
    hipLaunchKernelGGL(k_axpy_h4<false>, dim3(grid_of(np ? np : 1)), dim3(256), 0, stream, alpha, a, b, c, np, nvec);
  return launch_status();
}

vc_status vcb_axpy_bf16x4(float alpha, const uint16_t* a, const uint16_t* b, uint16_t* c, size_t nvec,
                          hipStream_t stream)
{
  return axpy_h4(true, alpha, a, b, c, nvec, stream);
}

vc_status vcb_axpy_f16x4(float alpha, const uint16_t* a, const uint16_t* b, uint16_t* c, size_t nvec,
                         hipStream_t stream)
{
  return axpy_h4(false, alpha, a, b, c, nvec, stream);
}

vc_status vcb_copy(const void* src, void* dst, size_t bytes, hipStream_t stream)
{
  if (bytes == 0) return VC_SUCCESS;
  if (!src || !dst) return VC_ERROR_INVALID_VALUE;
  if ((((uintptr_t)src | (uintptr_t)dst | bytes) & 15u) != 0) return VC_ERROR_MISALIGNED;
  hipLaunchKernelGGL(k_copy, dim3(grid_of(bytes / 16)), dim3(256), 0, stream, (const u32x4*)src, (u32x4*)dst,
                     bytes / 16);
  return launch_status();
}

}  // extern "C"
