// vc_stream.hip -- streaming kernels over compressed 3-vectors (gfx950).
//
// Every kernel is a memory stream: each wavefront reads and writes contiguous
// 1 KiB (or 3 KiB for float32 AoS) spans with 16-byte global loads/stores, and
// the whole codec (decode / FMA / encode) runs in registers between them.
//   k_axpy   : c = encode(alpha decode(a) + decode(b))    -- the C = A + B kernel of §5
//   k_encode : float32 AoS -> codes                        -- compress(), §3
//   k_decode : codes -> float32 AoS                        -- decompress(), Alg. (fr_fdiv_comp)
//   k_dot / k_norm2 : FP32 reductions over decoded vectors
#include <atomic>
#include <type_traits>

#include "vc_internal.hpp"

namespace vc {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool NT, class T>
__device__ __forceinline__ T ld(const T* p)
{
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st(T* p, T v)
{
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ------------------------------------------------------------------ axpy
// A tile is 2*BS*U consecutive codes.  Wave w of a block takes the U*128 codes from w*U*128 on:
// in step u lane l handles the pair at w*U*128 + u*128 + 2l, so every load/store instruction of
// a wave covers 1 KiB contiguous, and the steps of a lane are 1 KiB apart (immediate offsets of
// one scalar base plus one per-lane byte offset).
template <class L, int MODE, int PREC, int BS, int U, bool NT, bool DUMP, int TDEG = 15>
__global__ __launch_bounds__(BS) void k_axpy(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                             uint64_t* __restrict__ c, size_t n, uint32_t ntiles, float alpha,
                                             Params P0, float* __restrict__ dump)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
  // tiles [0, ntiles) take the 16-byte path (pointers 16-byte aligned); the rest is scalar
  constexpr size_t TILE = (size_t)2 * BS * U;
  const uint32_t first = (threadIdx.x >> 6) * (U * 128u) + 2u * (threadIdx.x & 63u);   // code index in a tile
  const uint32_t off = 8u * first;                                                      // its byte offset
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const size_t t0 = (size_t)tile * TILE;
    const u64x2* pa = (const u64x2*)((const char*)(a + t0) + off);
    const u64x2* pb = (const u64x2*)((const char*)(b + t0) + off);
    u64x2* pc = (u64x2*)((char*)(c + t0) + off);
    u64x2 va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      va[u] = ld<NT>(pa + 64 * u);
      vb[u] = ld<NT>(pb + 64 * u);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      u64x2 out;
#pragma unroll
      for (int h = 0; h < 2; h++) {
        float ax, ay, az, bx, by, bz;
        decode_vec<L, MODE, true>(va[u][h], P, ax, ay, az);
        decode_vec<L, MODE, true>(vb[u][h], P, bx, by, bz);
        if (special_code<L>(va[u][h]) || special_code<L>(vb[u][h])) {   // zero or reserved codes (rare)
          decode_vec<L, MODE>(va[u][h], P, ax, ay, az);
          decode_vec<L, MODE>(vb[u][h], P, bx, by, bz);
        }
        const float cx = __builtin_fmaf(alpha, ax, bx);
        const float cy = __builtin_fmaf(alpha, ay, by);
        const float cz = __builtin_fmaf(alpha, az, bz);
        if constexpr (DUMP) {
          const size_t i = t0 + first + (size_t)u * 128 + h;
          dump[3 * i] = cx; dump[3 * i + 1] = cy; dump[3 * i + 2] = cz;
        }
        out[h] = encode_vec<L, MODE, PREC, TDEG>(cx, cy, cz, P);
      }
      st<NT>(pc + 64 * u, out);
    }
  }
  // tail: vectors from ntiles*TILE on, one per thread
  const size_t start = (size_t)ntiles * TILE;
  for (size_t i = start + (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
    float ax, ay, az, bx, by, bz;
    decode_vec<L, MODE>(a[i], P, ax, ay, az);
    decode_vec<L, MODE>(b[i], P, bx, by, bz);
    const float cx = __builtin_fmaf(alpha, ax, bx);
    const float cy = __builtin_fmaf(alpha, ay, by);
    const float cz = __builtin_fmaf(alpha, az, bz);
    if constexpr (DUMP) { dump[3 * i] = cx; dump[3 * i + 1] = cy; dump[3 * i + 2] = cz; }
    c[i] = encode_vec<L, MODE, PREC, TDEG>(cx, cy, cz, P);
  }
  });
}

// ------------------------------------------------------------------ encode / decode
template <class L, int MODE, int PREC, int BS, int TDEG = 15>
__global__ __launch_bounds__(BS) void k_encode1(const float* __restrict__ xyz, uint64_t* __restrict__ codes,
                                                size_t n, Params P0)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS)
    codes[i] = encode_vec<L, MODE, PREC, TDEG>(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], P);
  });
}

// Encode and decode in wave tiles of 256 vectors, so that every load and store instruction of a
// wave covers 1 KiB contiguous: lane l holds codes 2l, 2l+1 and 128 + 2l, 129 + 2l (two 16-byte
// accesses), and the float32 AoS side (3 KiB per tile) passes through LDS (3 KiB per wave) as
// three 16-byte accesses per lane.  Requires 16-byte aligned pointers (checked by the launcher,
// which otherwise uses the one-vector-per-lane kernels); the tail past the last whole tile is
// done one vector per lane.
template <class L, int MODE, int BS, bool NT>
__global__ __launch_bounds__(BS) void k_decode_w(const uint64_t* __restrict__ codes, float* __restrict__ xyz,
                                                 size_t n, Params P0)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
  __shared__ float stage[BS / 64][256 * 3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* sw = stage[wv];
  const size_t ntile = n / 256;
  for (size_t t = (size_t)blockIdx.x * (BS / 64) + wv; t < ntile; t += (size_t)gridDim.x * (BS / 64)) {
    const u64x2* src = (const u64x2*)(codes + 256 * t);
    const u64x2 w0 = ld<NT>(src + lane), w1 = ld<NT>(src + 64 + lane);
    float v[12];
    decode_vec<L, MODE>(w0[0], P, v[0], v[1], v[2]);
    decode_vec<L, MODE>(w0[1], P, v[3], v[4], v[5]);
    decode_vec<L, MODE>(w1[0], P, v[6], v[7], v[8]);
    decode_vec<L, MODE>(w1[1], P, v[9], v[10], v[11]);
#pragma unroll
    for (int i = 0; i < 6; i++) { sw[6 * lane + i] = v[i]; sw[384 + 6 * lane + i] = v[6 + i]; }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f32x4* dst = (f32x4*)(xyz + 768 * t);
#pragma unroll
    for (int k = 0; k < 3; k++) st<NT>(dst + 64 * k + lane, *(const f32x4*)(sw + 4 * (64 * k + lane)));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  for (size_t i = 256 * ntile + (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS)
    decode_vec<L, MODE>(codes[i], P, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
  });
}

template <class L, int MODE, int PREC, int BS, bool NT, int TDEG = 15>
__global__ __launch_bounds__(BS) void k_encode_w(const float* __restrict__ xyz, uint64_t* __restrict__ codes,
                                                 size_t n, Params P0)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
  __shared__ float stage[BS / 64][256 * 3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* sw = stage[wv];
  const size_t ntile = n / 256;
  for (size_t t = (size_t)blockIdx.x * (BS / 64) + wv; t < ntile; t += (size_t)gridDim.x * (BS / 64)) {
    const f32x4* src = (const f32x4*)(xyz + 768 * t);
    f32x4 q[3];
#pragma unroll
    for (int k = 0; k < 3; k++) q[k] = ld<NT>(src + 64 * k + lane);
#pragma unroll
    for (int k = 0; k < 3; k++) *(f32x4*)(sw + 4 * (64 * k + lane)) = q[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float v[12];
#pragma unroll
    for (int i = 0; i < 6; i++) { v[i] = sw[6 * lane + i]; v[6 + i] = sw[384 + 6 * lane + i]; }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    u64x2 o0, o1;
    o0[0] = encode_vec<L, MODE, PREC, TDEG>(v[0], v[1], v[2], P);
    o0[1] = encode_vec<L, MODE, PREC, TDEG>(v[3], v[4], v[5], P);
    o1[0] = encode_vec<L, MODE, PREC, TDEG>(v[6], v[7], v[8], P);
    o1[1] = encode_vec<L, MODE, PREC, TDEG>(v[9], v[10], v[11], P);
    u64x2* dst = (u64x2*)(codes + 256 * t);
    st<NT>(dst + lane, o0);
    st<NT>(dst + 64 + lane, o1);
  }
  for (size_t i = 256 * ntile + (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS)
    codes[i] = encode_vec<L, MODE, PREC, TDEG>(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], P);
  });
}

template <class L, int MODE, int BS>
__global__ __launch_bounds__(BS) void k_decode1(const uint64_t* __restrict__ codes, float* __restrict__ xyz,
                                                size_t n, Params P0)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS)
    decode_vec<L, MODE>(codes[i], P, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
  });
}

// ------------------------------------------------------------------ reductions
template <int BS>
__device__ __forceinline__ float block_sum(float v)
{
  __shared__ float red[BS / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.0f;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / 64; i++) s += red[i];
  }
  return s;
}

template <class L, int MODE, int BS>
__global__ __launch_bounds__(BS) void k_dot(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                            size_t n, Params P, float* __restrict__ parts)
{
  float acc = 0.0f;
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
    acc += dot_pair<L, MODE>(a[i], b[i], P);
  }
  const float s = block_sum<BS>(acc);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

template <class L, int MODE, int BS>
__global__ __launch_bounds__(BS) void k_norm2(const uint64_t* __restrict__ a, size_t n, Params P,
                                              float* __restrict__ parts)
{
  float acc = 0.0f;
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
    const float r = decode_mag_checked<L, MODE>(a[i], P);
    acc = __builtin_fmaf(r, r, acc);
  }
  const float s = block_sum<BS>(acc);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// fixed-order final sum of the per-block partials (deterministic)
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ parts, int nparts,
                                                      float* __restrict__ out)
{
  float acc = 0.0f;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += parts[i];
  const float s = block_sum<256>(acc);
  if (threadIdx.x == 0) out[0] = s;
}

// ------------------------------------------------------------------ launchers
static inline unsigned grid_for(size_t work, size_t per_block, unsigned cap)
{
  size_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---- launch configuration of the streaming axpy per encoder precision (indexed by Prec), set by
// the autotuner; defaults are the fastest configurations measured at N = 2^27 on MI355X.  Each is
// one atomic word (block | vpt << 12 | nt << 20), so that a configuration change may race with
// launches on other threads: a launch uses the configuration current when it reads it.
static constexpr uint32_t pack_cfg(int block, int vpt, int nt)
{
  return (uint32_t)block | (uint32_t)vpt << 12 | (uint32_t)nt << 20;
}
static std::atomic<uint32_t> g_axpy_cfg[2] = {pack_cfg(512, 1, 1) /* PREC_F32 */, pack_cfg(256, 4, 1) /* PREC_F64 */};

StreamCfg stream_cfg(int prec)
{
  const uint32_t v = g_axpy_cfg[prec == PREC_F64 ? 1 : 0].load(std::memory_order_relaxed);
  return {(int)(v & 0xfffu), (int)((v >> 12) & 0xffu), (int)((v >> 20) & 1u)};
}

vc_status set_axpy_cfg(int prec, int block, int vpt, int nt)
{
  const bool okb = block == 128 || block == 256 || block == 512;
  const bool oku = vpt == 1 || vpt == 2 || (vpt == 4 && block >= 256);   // grid steps of 2 codes per lane
  if (!okb || !oku || (nt != 0 && nt != 1) || prec < -1 || prec > 1) return VC_ERROR_UNSUPPORTED_CODEC;
  for (int p = 0; p < 2; p++)
    if (prec < 0 || prec == p) g_axpy_cfg[p].store(pack_cfg(block, vpt, nt), std::memory_order_relaxed);
  return VC_SUCCESS;
}

template <class L, int MODE, int PREC, int BS, int U, bool NT>
static vc_status axpy_launch(const Resolved& R, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* c,
                             size_t n, float* dump, hipStream_t s)
{
  constexpr size_t TILE = (size_t)2 * BS * U;
  const bool aligned = (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15u) == 0;
  // tiles are counted in 32 bits: at most 2^31 of them (2^40 codes and more, beyond any HBM), so
  // that tile + grid (grid <= 2^30) cannot wrap; past that count the one-vector-per-lane tail
  // would take the rest
  const size_t ntiles = aligned ? (n / TILE < 0x80000000u ? n / TILE : 0x80000000u) : 0;
  const unsigned grid = grid_for(n, TILE, 1u << 30);
  // the tanh map's encoder evaluates the polynomial degree the fit needs (two instantiations)
  const bool low = MODE == TANH && PREC == PREC_F64 && tanh_tdeg(R.P.wdeg64) == 8;
  if (dump) {
    if (low)
      hipLaunchKernelGGL((k_axpy<L, MODE, PREC, BS, U, false, true, 8>), dim3(grid), dim3(BS), 0, s, a, b, c, n,
                         (uint32_t)ntiles, alpha, R.P, dump);
    else
      hipLaunchKernelGGL((k_axpy<L, MODE, PREC, BS, U, false, true>), dim3(grid), dim3(BS), 0, s, a, b, c, n,
                         (uint32_t)ntiles, alpha, R.P, dump);
  } else {
    if (low)
      hipLaunchKernelGGL((k_axpy<L, MODE, PREC, BS, U, NT, false, 8>), dim3(grid), dim3(BS), 0, s, a, b, c, n,
                         (uint32_t)ntiles, alpha, R.P, dump);
    else
      hipLaunchKernelGGL((k_axpy<L, MODE, PREC, BS, U, NT, false>), dim3(grid), dim3(BS), 0, s, a, b, c, n,
                         (uint32_t)ntiles, alpha, R.P, dump);
  }
  return launch_status();
}

template <class L, int MODE, int PREC>
static vc_status axpy_t(const Resolved& R, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* c,
                        size_t n, float* dump, hipStream_t s)
{
  // tuned variants for the default layout and uniform quantisation; other codecs use the shape the
  // tuner picks for that one, 256 x 4 steps of 2 vectors, NT (over 512 x 2 and 256 x 2: the same
  // codes, 1-4 % faster for the fractional-split, companded and truncating codecs)
  if constexpr (std::is_same<L, L0722>::value && MODE == PLAIN) {
    const StreamCfg g = stream_cfg(PREC);
    const int key = (g.block == 128 ? 0 : g.block == 256 ? 1 : 2) * 6 + (g.vpt == 4 ? 4 : g.vpt == 2 ? 2 : 0) + g.nt;
    switch (key) {
      case 0: return axpy_launch<L, MODE, PREC, 128, 1, false>(R, alpha, a, b, c, n, dump, s);
      case 1: return axpy_launch<L, MODE, PREC, 128, 1, true>(R, alpha, a, b, c, n, dump, s);
      case 2: return axpy_launch<L, MODE, PREC, 128, 2, false>(R, alpha, a, b, c, n, dump, s);
      case 3: return axpy_launch<L, MODE, PREC, 128, 2, true>(R, alpha, a, b, c, n, dump, s);
      case 6: return axpy_launch<L, MODE, PREC, 256, 1, false>(R, alpha, a, b, c, n, dump, s);
      case 7: return axpy_launch<L, MODE, PREC, 256, 1, true>(R, alpha, a, b, c, n, dump, s);
      case 8: return axpy_launch<L, MODE, PREC, 256, 2, false>(R, alpha, a, b, c, n, dump, s);
      case 9: return axpy_launch<L, MODE, PREC, 256, 2, true>(R, alpha, a, b, c, n, dump, s);
      case 10: return axpy_launch<L, MODE, PREC, 256, 4, false>(R, alpha, a, b, c, n, dump, s);
      case 11: return axpy_launch<L, MODE, PREC, 256, 4, true>(R, alpha, a, b, c, n, dump, s);
      case 12: return axpy_launch<L, MODE, PREC, 512, 1, false>(R, alpha, a, b, c, n, dump, s);
      case 13: return axpy_launch<L, MODE, PREC, 512, 1, true>(R, alpha, a, b, c, n, dump, s);
      case 14: return axpy_launch<L, MODE, PREC, 512, 2, false>(R, alpha, a, b, c, n, dump, s);
      case 15: return axpy_launch<L, MODE, PREC, 512, 2, true>(R, alpha, a, b, c, n, dump, s);
      case 16: return axpy_launch<L, MODE, PREC, 512, 4, false>(R, alpha, a, b, c, n, dump, s);
      default: return axpy_launch<L, MODE, PREC, 512, 4, true>(R, alpha, a, b, c, n, dump, s);
    }
  } else {
    return axpy_launch<L, MODE, PREC, 256, 4, true>(R, alpha, a, b, c, n, dump, s);
  }
}

template <class L, int MODE, int PREC, int TDEG>
static vc_status encode_d(const Resolved& R, const float* xyz, uint64_t* codes, size_t n, hipStream_t s)
{
  constexpr int BS = 256;
  const bool aligned = (((uintptr_t)xyz | (uintptr_t)codes) & 15u) == 0;
  if (aligned) {
    const unsigned grid = grid_for(n, (size_t)4 * BS, 1u << 30);
    hipLaunchKernelGGL((k_encode_w<L, MODE, PREC, BS, true, TDEG>), dim3(grid), dim3(BS), 0, s, xyz, codes, n, R.P);
  } else {
    const unsigned grid = grid_for(n, (size_t)BS, 1u << 30);
    hipLaunchKernelGGL((k_encode1<L, MODE, PREC, BS, TDEG>), dim3(grid), dim3(BS), 0, s, xyz, codes, n, R.P);
  }
  return launch_status();
}

template <class L, int MODE, int PREC>
static vc_status encode_t(const Resolved& R, const float* xyz, uint64_t* codes, size_t n, hipStream_t s)
{
  if (MODE == TANH && PREC == PREC_F64 && tanh_tdeg(R.P.wdeg64) == 8)
    return encode_d<L, MODE, PREC, 8>(R, xyz, codes, n, s);
  return encode_d<L, MODE, PREC, 15>(R, xyz, codes, n, s);
}

template <class L, int MODE, int PREC>
static vc_status decode_t(const Resolved& R, const uint64_t* codes, float* xyz, size_t n, hipStream_t s)
{
  constexpr int BS = 256;
  const bool aligned = (((uintptr_t)xyz | (uintptr_t)codes) & 15u) == 0;
  if (aligned) {
    const unsigned grid = grid_for(n, (size_t)4 * BS, 1u << 30);
    hipLaunchKernelGGL((k_decode_w<L, MODE, BS, true>), dim3(grid), dim3(BS), 0, s, codes, xyz, n, R.P);
  } else {
    const unsigned grid = grid_for(n, (size_t)BS, 1u << 30);
    hipLaunchKernelGGL((k_decode1<L, MODE, BS>), dim3(grid), dim3(BS), 0, s, codes, xyz, n, R.P);
  }
  return launch_status();
}

int reduce_parts(size_t n)
{
  size_t g = (n + 256 * 16 - 1) / (256 * 16);
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return (int)g;
}

template <class L, int MODE, int PREC>
static vc_status dot_t(const Resolved& R, const uint64_t* a, const uint64_t* b, size_t n, float* parts, int np,
                       float* out, hipStream_t s)
{
  hipLaunchKernelGGL((k_dot<L, MODE, 256>), dim3(np), dim3(256), 0, s, a, b, n, R.P, parts);
  vc_status st = launch_status();
  if (st != VC_SUCCESS) return st;
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, (const float*)parts, np, out);
  return launch_status();
}

template <class L, int MODE, int PREC>
static vc_status norm2_t(const Resolved& R, const uint64_t* a, size_t n, float* parts, int np, float* out,
                         hipStream_t s)
{
  hipLaunchKernelGGL((k_norm2<L, MODE, 256>), dim3(np), dim3(256), 0, s, a, n, R.P, parts);
  vc_status st = launch_status();
  if (st != VC_SUCCESS) return st;
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, (const float*)parts, np, out);
  return launch_status();
}

vc_status launch_axpy(const Resolved& R, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* c,
                      size_t n, float* dump, hipStream_t s)
{
  VC_DISPATCH(R, axpy_t, R, alpha, a, b, c, n, dump, s);
}

vc_status launch_encode(const Resolved& R, const float* xyz, uint64_t* codes, size_t n, hipStream_t s)
{
  VC_DISPATCH(R, encode_t, R, xyz, codes, n, s);
}

vc_status launch_decode(const Resolved& R, const uint64_t* codes, float* xyz, size_t n, hipStream_t s)
{
  VC_DISPATCH_NOPREC(R, decode_t, R, codes, xyz, n, s);
}

vc_status launch_dot(const Resolved& R, const uint64_t* a, const uint64_t* b, size_t n, float* parts, int np,
                     float* out, hipStream_t s)
{
  VC_DISPATCH_NOPREC(R, dot_t, R, a, b, n, parts, np, out, s);
}

vc_status launch_norm2(const Resolved& R, const uint64_t* a, size_t n, float* parts, int np, float* out,
                       hipStream_t s)
{
  VC_DISPATCH_NOPREC(R, norm2_t, R, a, n, parts, np, out, s);
}

}  // namespace vc
