// vc_apply.hip -- fused decode + dense operator apply on the matrix cores (gfx950).
//
// For each element e: out[e] (rows x 3) = M (rows x cols) . X_e, X_e[k] = decode(U[e][k]).
// This is the operator pattern of Alg. (fr_fdiv_comp) -- a small dense operator applied to
// compressed nodal vectors -- written as one batched GEMM  Out (rows x 3E) = M (rows x K) .
// [X_1 | ... | X_E] (K x 3E), K = cols, with the right-hand side decoded on the fly.
//
// MFMA tiling (v_mfma_f32_16x16x4f32, FP32 in, FP32 accumulate):
//   * a wave owns 16 elements; their x, y and z components form three 16-column B tiles;
//   * rows are covered by MT 16-row tiles, so a wave keeps 3 MT accumulators (4 registers each);
//   * K is interleaved: at step s lane l (element e0 + l%16, quarter q = l/16) takes operand row
//     k = 4s + q, so the four quarters of one element read 32 contiguous bytes of its codes; each
//     lane decodes exactly one code per step and feeds x, y, z straight into the B fragments.
//     The next step's code is loaded before the current step's MFMAs (software pipelining);
//     operand rows k >= cols and elements past the end use the zero code, which decodes to 0;
//   * M is staged once per workgroup in LDS, transposed (A[k][row], row stride RS = rows rounded
//     up to 24 mod 32 words, so the four quarters hit different banks); rows beyond `rows` are
//     read clamped and never stored;
//   * the results leave through LDS: a lane's accumulators are 4 rows of one element, which
//     written directly make 64 scattered 12-byte pieces per store; staged per 16-row block, each
//     element's rows are contiguous and consecutive lanes store consecutive 8-byte pairs.
// A workgroup is 8 waves (128 elements per step) sharing one copy of M, one workgroup per CU,
// persistent over the element tiles (the last, partial round spread over the CUs).
#include "vc_internal.hpp"

namespace vc {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int APPLY_WAVES = 8;
constexpr int APPLY_EPW = 16;      // elements per wave

// A load the optimiser keeps where it is written (a relaxed wavefront-scope atomic load is an
// ordinary global load, but it is not sunk to its use, so it stays one K-step ahead)
__device__ __forceinline__ uint64_t ld_keep(const uint64_t* p)
{
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// LDS row stride: >= rows and == 24 (mod 32) words
inline __host__ __device__ int apply_rs(int rows) { return rows + ((24 - rows % 32) + 32) % 32; }

template <class L, int MODE, int MT>
__global__ __launch_bounds__(64 * APPLY_WAVES) void k_apply(const float* __restrict__ M, int rows, int cols,
                                                              int KS, int RS, const uint64_t* __restrict__ U,
                                                              float* __restrict__ out, size_t n_elem, int pairs,
                                                              Params P)
{
  extern __shared__ float As[];  // [4*KS][RS], transposed, zero for k >= cols; then per-wave staging
  const int KP = 4 * KS;
  for (int i = threadIdx.x; i < KP * RS; i += blockDim.x) {
    const int k = i / RS, r = i - k * RS;
    As[i] = (k < cols && r < rows) ? M[(size_t)r * cols + k] : 0.0f;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j = lane & 15;        // column within a tile = element within the wave's 16
  const int q = lane >> 4;        // K quarter
  // Tiles: R full rounds in which wave w of workgroup b takes tile i W + 8 b + w (W waves in
  // all), then the rem = ntiles mod W left over go one per wave in the order (w, b) = (0, 0),
  // (0, 1), ...: waves 0-3 of every workgroup before any wave 4-7, so the last round spreads
  // over as many CUs and SIMDs as it can instead of filling a few CUs with 8 waves each.
  const size_t ntiles = (n_elem + APPLY_EPW - 1) / APPLY_EPW;
  const size_t W = (size_t)gridDim.x * APPLY_WAVES;
  const size_t R = ntiles / W, rem = ntiles - R * W;
  const size_t kx = (size_t)wave * gridDim.x + blockIdx.x;     // this wave's rank in the last round
  const size_t mine = R + (kx < rem ? 1 : 0);
  for (size_t i = 0; i < mine; i++) {
    const size_t t = i < R ? i * W + (size_t)blockIdx.x * APPLY_WAVES + wave : R * W + kx;
    const size_t e = t * APPLY_EPW + j;
    const bool e_ok = e < n_elem;
    const uint64_t* Ue = U + (e_ok ? e : 0) * (size_t)cols;
    f32x4 acc[MT][3];
#pragma unroll
    for (int m = 0; m < MT; m++)
#pragma unroll
      for (int c = 0; c < 3; c++) acc[m][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // the code of step s + 1 is loaded while step s multiplies (from a clamped, always valid
    // address; its validity is applied where it is used)
    int kn = q;
    uint64_t wraw = ld_keep(Ue + (kn < cols ? kn : cols - 1));
    bool wok = e_ok && kn < cols;
    for (int s = 0; s < KS; s++) {
      const int k = kn;
      const uint64_t w = wok ? wraw : 0ull;      // the zero code decodes to (0, 0, 0)
      kn += 4;
      wraw = ld_keep(Ue + (kn < cols ? kn : cols - 1));
      wok = e_ok && kn < cols;
      float bx, by, bz;
      decode_vec<L, MODE>(w, P, bx, by, bz);
      const float* Ak = As + k * RS;
      float a[MT];
#pragma unroll
      for (int m = 0; m < MT; m++) {
        const int r = 16 * m + j;                 // rows past the end are read clamped, never stored
        a[m] = Ak[r < rows ? r : rows - 1];
      }
#pragma unroll
      for (int m = 0; m < MT; m++) acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], bx, acc[m][0], 0, 0, 0);
#pragma unroll
      for (int m = 0; m < MT; m++) acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], by, acc[m][1], 0, 0, 0);
#pragma unroll
      for (int m = 0; m < MT; m++) acc[m][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], bz, acc[m][2], 0, 0, 0);
    }
    // D[i][jj] at lane jj + 16 (i/4), register i%4: this lane holds rows 16m + 4q + (0..3) of
    // element e, for the three components.  Each 16-row block is staged through this wave's LDS
    // area as 16 element blocks of 48 floats and written back with consecutive lanes on
    // consecutive 8-byte pairs (an element's block of rows is contiguous in `out`).
    float* st = As + KP * RS + wave * (16 * 48);
    const size_t t0 = t * APPLY_EPW;
#pragma unroll
    for (int m = 0; m < MT; m++) {
#pragma unroll
      for (int rr = 0; rr < 4; rr++)
#pragma unroll
        for (int c = 0; c < 3; c++) st[j * 48 + (4 * q + rr) * 3 + c] = acc[m][c][rr];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int nr = rows - 16 * m < 16 ? rows - 16 * m : 16;   // rows of this block (>= 1)
      if (nr == 16 && pairs) {
#pragma unroll
        for (int i = 0; i < 6; i++) {
          const int f2 = i * 64 + lane;             // pair index over 16 elements x 24 pairs
          const int el = f2 / 24, off = 2 * (f2 - el * 24);
          const size_t eg = t0 + el;
          if (eg < n_elem) {
            const float2 v = *(const float2*)(st + el * 48 + off);
            *(float2*)(out + eg * (size_t)rows * 3 + 48 * m + off) = v;
          }
        }
      } else {
        const int nb = 3 * nr;
        for (int f = lane; f < 16 * nb; f += 64) {
          const int el = f / nb, off = f - el * nb;
          const size_t eg = t0 + el;
          if (eg < n_elem) out[eg * (size_t)rows * 3 + 48 * m + off] = st[el * 48 + off];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

template <class L, int MODE, int MT>
static vc_status apply_mt(const Resolved& R, const float* M, int rows, int cols, const uint64_t* U, float* out,
                          size_t n_elem, hipStream_t s)
{
  const int KS = (cols + 3) / 4;
  const int RS = apply_rs(rows);
  const size_t lds = ((size_t)4 * KS * RS + (size_t)APPLY_WAVES * 16 * 48) * sizeof(float);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  const size_t ntiles = (n_elem + APPLY_EPW - 1) / APPLY_EPW;
  size_t grid = (ntiles + APPLY_WAVES - 1) / APPLY_WAVES;
  const size_t cap = (size_t)ncu;                   // one resident workgroup per CU
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_apply<L, MODE, MT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
    return VC_ERROR_HIP;
  // 8-byte stores need an even row length (3 rows) and an 8-byte aligned output
  const int pairs = (rows % 2 == 0) && (((uintptr_t)out & 7u) == 0);
  hipLaunchKernelGGL((k_apply<L, MODE, MT>), dim3((unsigned)grid), dim3(64 * APPLY_WAVES), lds, s, M, rows, cols,
                     KS, RS, U, out, n_elem, pairs, R.P);
  return launch_status();
}

template <class L, int MODE>
static vc_status apply_t(const Resolved& R, const float* M, int rows, int cols, const uint64_t* U, float* out,
                         size_t n_elem, hipStream_t s)
{
  switch ((rows + 15) / 16) {
#define VC_MT(n) case n: return apply_mt<L, MODE, n>(R, M, rows, cols, U, out, n_elem, s);
    VC_MT(1) VC_MT(2) VC_MT(3) VC_MT(4) VC_MT(5) VC_MT(6) VC_MT(7) VC_MT(8)
    VC_MT(9) VC_MT(10) VC_MT(11) VC_MT(12) VC_MT(13) VC_MT(14) VC_MT(15) VC_MT(16)
#undef VC_MT
    default: return VC_ERROR_INVALID_VALUE;
  }
}

vc_status launch_apply(const Resolved& R, const float* M, int rows, int cols, const uint64_t* U, float* out,
                       size_t n_elem, hipStream_t s)
{
  switch (R.layout * 4 + R.mode) {
    case 0: return apply_t<L0722, PLAIN>(R, M, rows, cols, U, out, n_elem, s);
    case 3: return apply_t<L0722, FRAC>(R, M, rows, cols, U, out, n_elem, s);
    case 4: return apply_t<L0723, PLAIN>(R, M, rows, cols, U, out, n_elem, s);
    case 8: return apply_t<L0823, PLAIN>(R, M, rows, cols, U, out, n_elem, s);
    case 12: return apply_t<L1823, PLAIN>(R, M, rows, cols, U, out, n_elem, s);
    default: return VC_ERROR_UNSUPPORTED_CODEC;
  }
}

}  // namespace vc

using namespace vc;

extern "C" vc_status vc_fused_apply(const vc_codec* c, const float* M, int rows, int cols, const uint64_t* U,
                                    float* out, size_t n_elem, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (rows < 1 || rows > 256 || cols < 1 || cols > 256) return VC_ERROR_INVALID_VALUE;
  // M^T staged in LDS: 4 ceil(cols/4) x RS floats must fit one workgroup's 80 KiB share
  if ((size_t)4 * ((cols + 3) / 4) * apply_rs(rows) * sizeof(float) > 80 * 1024) return VC_ERROR_INVALID_VALUE;
  if (n_elem == 0) return VC_SUCCESS;
  if (!M || !U || !out) return VC_ERROR_INVALID_VALUE;
  if (((uintptr_t)M & 3u) || ((uintptr_t)U & 7u) || ((uintptr_t)out & 3u)) return VC_ERROR_MISALIGNED;
  return launch_apply(R, M, rows, cols, U, out, n_elem, stream);
}
