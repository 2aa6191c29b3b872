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
//     written directly make 64 scattered 12-byte pieces per store.  Where LDS has room (WHOLE),
//     each wave stages 4 complete elements at a time, the image of 4 x rows x 3 contiguous floats
//     of `out`, and writes it with 16-byte stores, every store instruction 1 KiB contiguous;
//     otherwise it stages one 16-row block of its 16 elements at a time and consecutive lanes
//     store consecutive 8-byte pairs of each element's 192-byte run.
// A workgroup is 8 waves (128 elements per step) sharing one copy of M, one workgroup per CU,
// persistent over the element tiles (the last, partial round spread over the CUs).
#include <atomic>

#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int APPLY_WAVES = 8;
constexpr int APPLY_EPW = 16;      // elements per wave
constexpr int APPLY_AHEAD = 4;     // K-steps whose codes are in flight ahead of their use
constexpr int APPLY_MTC = 2;       // row blocks per unit of work in the last, partial round

// which matrix cores the apply uses (vcx_set_apply_mode)
static std::atomic<int> g_apply_mode{VCX_APPLY_AUTO};

// A load the optimiser keeps where it is written (a relaxed wavefront-scope atomic load is an
// ordinary global load, but it is not sunk to its use, so it stays one K-step ahead)
__device__ __forceinline__ uint64_t ld_keep(const uint64_t* p)
{
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// LDS row stride: >= rows and == 24 (mod 32) words
inline __host__ __device__ int apply_rs(int rows) { return rows + ((24 - rows % 32) + 32) % 32; }

// floats of per-wave output staging: 4 whole elements, or one 16-row block of 16 elements (the
// row-block stores of the last tiles use the whole-element area too)
inline __host__ __device__ int apply_stage(bool whole, int rows)
{
  return whole && 12 * rows > 16 * 48 ? 12 * rows : 16 * 48;
}

// One tile's products: acc[m] = rows 16 (m0 + m) .. 16 (m0 + m) + 15 of M . X over all K, for the
// 16 elements of the tile (lane: element j, K quarter q).  Rows past `rows` are computed from
// clamped operator reads and never stored.
template <class L, int MODE, int NM>
__device__ __forceinline__ void tile_mma(f32x4 (&acc)[NM][3], const float* As, int RS, int KS, int rows, int cols,
                                         const uint64_t* __restrict__ Ue, bool e_ok, int j, int q, int m0,
                                         const Params& P)
{
#pragma unroll
  for (int m = 0; m < NM; m++)
#pragma unroll
    for (int c = 0; c < 3; c++) acc[m][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // The codes of the next APPLY_AHEAD steps are in flight while step s multiplies: a ring of
  // registers, slot d holding the code of the steps d, d + APPLY_AHEAD, ... (loaded from a
  // clamped, always valid address).  A lane whose operand row is past `cols`, or whose element
  // is past the end, uses the zero code instead, which decodes to (0, 0, 0).
  uint64_t ring[APPLY_AHEAD];
#pragma unroll
  for (int d = 0; d < APPLY_AHEAD; d++) {
    const int k = 4 * d + q;
    ring[d] = ld_keep(Ue + (k < cols ? k : cols - 1));
  }
  for (int s0 = 0; s0 < KS; s0 += APPLY_AHEAD) {
#pragma unroll
    for (int d = 0; d < APPLY_AHEAD; d++) {
      const int s = s0 + d;
      if (s >= KS) break;                       // uniform
      const int k = 4 * s + q;
      const uint64_t w = (e_ok && k < cols) ? ring[d] : 0ull;
      const int kn = k + 4 * APPLY_AHEAD;
      ring[d] = ld_keep(Ue + (kn < cols ? kn : cols - 1));
      float bx, by, bz;
      decode_vec<L, MODE>(w, P, bx, by, bz);
      const float* Ak = As + k * RS;
      float a[NM];
#pragma unroll
      for (int m = 0; m < NM; m++) {
        const int r = 16 * (m0 + m) + j;
        a[m] = Ak[r < rows ? r : rows - 1];
      }
#pragma unroll
      for (int m = 0; m < NM; m++) acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], bx, acc[m][0], 0, 0, 0);
#pragma unroll
      for (int m = 0; m < NM; m++) acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], by, acc[m][1], 0, 0, 0);
#pragma unroll
      for (int m = 0; m < NM; m++) acc[m][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], bz, acc[m][2], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void wave_lds_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// D[i][jj] at lane jj + 16 (i/4), register i%4: a lane holds rows 16m + 4q + (0..3) of element j
// for the three components.
//
// Whole tiles: elements 4g .. 4g+3 (the lanes with j / 4 == g) are staged as their image in
// `out`, [4][rows][3]; it starts 48 rows g bytes past the tile, so with `out` 16-byte aligned the
// wave writes it with aligned 16-byte stores, each store instruction 1 KiB contiguous.
template <int MT>
__device__ __forceinline__ void store_whole(const f32x4 (&acc)[MT][3], float* st, float* __restrict__ out, int rows,
                                            size_t t0, size_t n_elem, int lane, int j, int q)
{
  const int nf = 12 * rows;                          // floats of 4 elements
  for (int g = 0; g < 4; g++) {
    const size_t eg0 = t0 + 4 * g;
    if (eg0 >= n_elem) break;                        // uniform across the wave
    if ((j >> 2) == g) {
      float* se = st + (j & 3) * (3 * rows);
#pragma unroll
      for (int m = 0; m < MT; m++)
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
          const int r = 16 * m + 4 * q + rr;
          if (m < MT - 1 || r < rows)                // rows past the end are not staged
#pragma unroll
            for (int c = 0; c < 3; c++) se[3 * r + c] = acc[m][c][rr];
        }
    }
    wave_lds_sync();
    float* og = out + eg0 * (size_t)rows * 3;
    if (n_elem - eg0 >= 4) {
      const float4* s4 = (const float4*)st;
      float4* o4 = (float4*)og;
      for (int i = lane; i < nf / 4; i += 64) o4[i] = s4[i];
    } else {
      const int nv = (int)(n_elem - eg0) * 3 * rows;
      for (int i = lane; i < nv; i += 64) og[i] = st[i];
    }
    wave_lds_sync();
  }
}

// Row blocks m0 .. m0 + NM - 1 (those below `rows`) of the tile's 16 elements: each 16-row block
// is staged as 16 element blocks of 48 floats and written back with consecutive lanes on
// consecutive 8-byte pairs (an element's block of rows is contiguous in `out`).
template <int NM>
__device__ __forceinline__ void store_blocks(const f32x4 (&acc)[NM][3], float* st, float* __restrict__ out, int rows,
                                             size_t t0, size_t n_elem, int m0, int pairs, int lane, int j, int q)
{
#pragma unroll
  for (int m = 0; m < NM; m++) {
    const int mb = m0 + m;
    if (16 * mb >= rows) break;                      // uniform
#pragma unroll
    for (int rr = 0; rr < 4; rr++)
#pragma unroll
      for (int c = 0; c < 3; c++) st[j * 48 + (4 * q + rr) * 3 + c] = acc[m][c][rr];
    wave_lds_sync();
    const int nr = rows - 16 * mb < 16 ? rows - 16 * mb : 16;   // rows of this block (>= 1)
    if (nr == 16 && pairs) {
#pragma unroll
      for (int i = 0; i < 6; i++) {
        const int f2 = i * 64 + lane;               // pair index over 16 elements x 24 pairs
        const int el = f2 / 24, off = 2 * (f2 - el * 24);
        const size_t eg = t0 + el;
        if (eg < n_elem) {
          const float2 v = *(const float2*)(st + el * 48 + off);
          *(float2*)(out + eg * (size_t)rows * 3 + 48 * mb + off) = v;
        }
      }
    } else {
      const int nb = 3 * nr;
      for (int f = lane; f < 16 * nb; f += 64) {
        const int el = f / nb, off = f - el * nb;
        const size_t eg = t0 + el;
        if (eg < n_elem) out[eg * (size_t)rows * 3 + 48 * mb + off] = st[el * 48 + off];
      }
    }
    wave_lds_sync();
  }
}

template <class L, int MODE, int MT, bool WHOLE>
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
  float* st = As + KP * RS + wave * apply_stage(WHOLE, rows);
  // Tiles: R full rounds in which wave w of workgroup b takes tile i W + 8 b + w (W waves in
  // all).  The rem = ntiles mod W tiles left over are cut into units of APPLY_MTC row blocks
  // when that gives no wave more than one unit (else a unit is a whole tile), and the units go
  // one per wave in the order (w, b) = (0, 0), (0, 1), ...: waves 0-3 of every workgroup before
  // any wave 4-7, so the last round spreads over as many CUs and SIMDs as it can.
  const size_t ntiles = (n_elem + APPLY_EPW - 1) / APPLY_EPW;
  const size_t W = (size_t)gridDim.x * APPLY_WAVES;
  const size_t R = ntiles / W, rem = ntiles - R * W;
  const size_t kx = (size_t)wave * gridDim.x + blockIdx.x;     // this wave's rank in the last round
  for (size_t i = 0; i < R; i++) {
    const size_t t = i * W + (size_t)blockIdx.x * APPLY_WAVES + wave;
    const size_t e = t * APPLY_EPW + j;      // past the end only in the last tile (rem == 0)
    const bool e_ok = e < n_elem;
    f32x4 acc[MT][3];
    tile_mma<L, MODE, MT>(acc, As, RS, KS, rows, cols, U + (e_ok ? e : 0) * (size_t)cols, e_ok, j, q, 0, P);
    if constexpr (WHOLE)
      store_whole<MT>(acc, st, out, rows, t * APPLY_EPW, n_elem, lane, j, q);
    else
      store_blocks<MT>(acc, st, out, rows, t * APPLY_EPW, n_elem, 0, pairs, lane, j, q);
  }
  constexpr int MTC = MT < APPLY_MTC ? MT : APPLY_MTC;
  constexpr int NC = (MT + MTC - 1) / MTC;
  if (NC > 1 && rem * NC <= W) {
    for (size_t u = kx; u < rem * NC; u += W) {
      const size_t t = R * W + u / NC;
      const int m0 = (int)(u % NC) * MTC;
      const size_t e = t * APPLY_EPW + j;
      const bool e_ok = e < n_elem;
      f32x4 acc[MTC][3];
      tile_mma<L, MODE, MTC>(acc, As, RS, KS, rows, cols, U + (e_ok ? e : 0) * (size_t)cols, e_ok, j, q, m0, P);
      store_blocks<MTC>(acc, st, out, rows, t * APPLY_EPW, n_elem, m0, pairs, lane, j, q);
    }
  } else if (kx < rem) {
    const size_t t = R * W + kx;
    const size_t e = t * APPLY_EPW + j;
    const bool e_ok = e < n_elem;
    f32x4 acc[MT][3];
    tile_mma<L, MODE, MT>(acc, As, RS, KS, rows, cols, U + (e_ok ? e : 0) * (size_t)cols, e_ok, j, q, 0, P);
    if constexpr (WHOLE)
      store_whole<MT>(acc, st, out, rows, t * APPLY_EPW, n_elem, lane, j, q);
    else
      store_blocks<MT>(acc, st, out, rows, t * APPLY_EPW, n_elem, 0, pairs, lane, j, q);
  }
}

// ---------------------------------------------------------------- split-bf16 variant
// The same products on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16), with FP32 accuracy:
// every FP32 operand is split into three bf16 parts, x = x1 + x2 + x3 (x1 = bf16(x), x2 =
// bf16(x - x1), x3 = bf16(x - x1 - x2); the differences are exact in FP32, and x3 rounds off at
// most 2^-24 |x|), and a b is taken as the six part products with i + j <= 4:
//   a1 b1 + a1 b2 + a2 b1 + a1 b3 + a2 b2 + a3 b1,
// each exact in FP32 (8-bit by 8-bit significands) and accumulated in FP32 by the matrix core.
// The three dropped products are below 3 2^-24 |a| |b|, so each term is as accurate as one FP32
// product.  A bf16 MFMA of K = 32 takes half the cycles of an FP32 MFMA of K = 4 (16 against
// 32), so the six of them cover 8 times the K in 3 times the time: ~2.7x less matrix time.
//   * A (the operator) is split once per workgroup into LDS, part-major [3][rows][RK] bf16 with
//     K contiguous (RK = 32 KS + 8: the 16-byte pad spreads a wave's 16 rows over the banks);
//   * B: at K-step s lane l (element j = l % 16, quarter q = l / 16) decodes the 8 codes
//     k = 32 s + 8 q + i (64 contiguous bytes) and splits their x, y, z;
//   * a tile takes two passes over K, each for about half of its row blocks: the accumulators of
//     all blocks, the split operands and the decode do not fit the registers of two waves per
//     SIMD together (the second pass decodes the codes again, reading them from the L2);
//   * the accumulator layout is the FP32 kernel's, so the results leave through the same 16-row
//     block staging.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l)
{
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

// bf16 RNE of (a, b), packed: a in the low half (element 0), b in the high half
__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

// split3 of a pair of values, each part packed as it is formed: w[p] holds part p of (a, b)
__device__ __forceinline__ void split3_pair(float a, float b, uint32_t (&w)[3])
{
  w[0] = pk_bf16(a, b);
  const float ra = a - __uint_as_float(w[0] << 16), rb = b - __uint_as_float(w[0] & 0xffff0000u);
  w[1] = pk_bf16(ra, rb);
  const float sa = ra - __uint_as_float(w[1] << 16), sb = rb - __uint_as_float(w[1] & 0xffff0000u);
  w[2] = pk_bf16(sa, sb);
}

inline __host__ __device__ int apply_rk(int cols) { return 32 * ((cols + 31) / 32) + 8; }

template <class L, int MODE, int NM>
__device__ __forceinline__ void tile_mma_bf(f32x4 (&acc)[NM][3], const __bf16* Ab, int RK, int KS, int RA,
                                            int cols, const uint64_t* __restrict__ Ue, bool e_ok, int j, int q,
                                            int m0, const Params& P)
{
#pragma unroll
  for (int m = 0; m < NM; m++)
#pragma unroll
    for (int c = 0; c < 3; c++) acc[m][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const size_t pstride = (size_t)RA * RK;            // one part of A (RA rows, zero past `rows`)
  const __bf16* Aj = Ab + (size_t)(16 * m0 + j) * RK + 8 * q;
  for (int s = 0; s < KS; s++) {
    // the step's codes (clamped addresses; past `cols`, or past the end, the zero code is used)
    uint64_t cur[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const int k = 32 * s + 8 * q + i;
      cur[i] = ld_keep(Ue + (k < cols ? k : cols - 1));
    }
    // B[component][part]: K = 8 q .. 8 q + 7, dword d holding the codes 2d, 2d + 1 (a pair of
    // codes decoded and split at a time, each part packed as it is formed)
    uint32_t Bw[3][3][4];
#pragma unroll
    for (int d = 0; d < 4; d++) {
      float v[2][3];
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int k = 32 * s + 8 * q + 2 * d + h;
        const uint64_t w = (e_ok && k < cols) ? cur[2 * d + h] : 0ull;
        decode_vec<L, MODE>(w, P, v[h][0], v[h][1], v[h][2]);
      }
#pragma unroll
      for (int c = 0; c < 3; c++) {
        uint32_t wp[3];
        split3_pair(v[0][c], v[1][c], wp);
#pragma unroll
        for (int p = 0; p < 3; p++) Bw[c][p][d] = wp[p];
      }
    }
    bf16x8 B[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int p = 0; p < 3; p++) {
        typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
        B[c][p] = __builtin_bit_cast(bf16x8, (u32x4_t){Bw[c][p][0], Bw[c][p][1], Bw[c][p][2], Bw[c][p][3]});
      }
    // (scheduling fences: the operator parts of one pair of row blocks in registers at a time)
    __builtin_amdgcn_sched_barrier(0);
    // part products (i, j) with i + j <= 4, for pairs of row blocks (independent accumulators
    // between dependent MFMAs)
    constexpr int PA[6] = {0, 0, 1, 0, 1, 2}, PB[6] = {0, 1, 0, 2, 1, 0};
#pragma unroll
    for (int m = 0; m < NM; m += 2) {
      bf16x8 A[2][3];
#pragma unroll
      for (int mm = 0; mm < 2; mm++)
#pragma unroll
        for (int pa = 0; pa < 3; pa++)
          A[mm][pa] = (m + mm < NM) ? *(const bf16x8*)(Aj + pa * pstride + (size_t)(16 * (m + mm)) * RK + 32 * s)
                                    : A[0][pa];
#pragma unroll
      for (int t = 0; t < 6; t++)
#pragma unroll
        for (int mm = 0; mm < 2; mm++)
          if (m + mm < NM)
#pragma unroll
            for (int c = 0; c < 3; c++)
              acc[m + mm][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mm][PA[t]], B[c][PB[t]], acc[m + mm][c], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <class L, int MODE, int MT>
__global__ __launch_bounds__(64 * APPLY_WAVES) void k_apply_bf(const float* __restrict__ M, int rows, int cols,
                                                                 int KS, int RK, const uint64_t* __restrict__ U,
                                                                 float* __restrict__ out, size_t n_elem, int pairs,
                                                                 Params P)
{
  extern __shared__ float smem[];   // bf16 [3][16 MT][RK] (A split in parts), then per-wave staging
  __bf16* Ab = (__bf16*)smem;
  constexpr int RA = 16 * MT;      // rows padded to whole row blocks (zero rows are never stored)
  const size_t pstride = (size_t)RA * RK;
#pragma unroll 1
  for (int i = threadIdx.x; i < RA * RK; i += blockDim.x) {
    const int r = i / RK, k = i - r * RK;
    __bf16 h, m, l;
    split3(k < cols && r < rows ? M[(size_t)r * cols + k] : 0.0f, h, m, l);
    Ab[i] = h;
    Ab[pstride + i] = m;
    Ab[2 * pstride + i] = l;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j = lane & 15;
  const int q = lane >> 4;
  float* st = smem + (3 * pstride + 1) / 2 + wave * (16 * 48);   // after A (rounded up to a float)
  // tile schedule as in k_apply
  const size_t ntiles = (n_elem + APPLY_EPW - 1) / APPLY_EPW;
  const size_t W = (size_t)gridDim.x * APPLY_WAVES;
  const size_t R = ntiles / W, rem = ntiles - R * W;
  const size_t kx = (size_t)wave * gridDim.x + blockIdx.x;
  // a whole tile in two passes over K of about MT/2 row blocks each (the accumulators of all MT
  // blocks, the split operands and the decode do not fit the registers of two waves per SIMD
  // together); the second pass reads the tile's codes again, from the L2
  constexpr int NH = (MT + 1) / 2;
  auto half_tiles = [&](const uint64_t* Ue, bool e_ok, size_t t0) __attribute__((always_inline)) {
    {
      f32x4 acc[NH][3];
      tile_mma_bf<L, MODE, NH>(acc, Ab, RK, KS, RA, cols, Ue, e_ok, j, q, 0, P);
      store_blocks<NH>(acc, st, out, rows, t0, n_elem, 0, pairs, lane, j, q);
    }
    if constexpr (MT - NH > 0) {
      f32x4 acc[MT - NH][3];
      tile_mma_bf<L, MODE, MT - NH>(acc, Ab, RK, KS, RA, cols, Ue, e_ok, j, q, NH, P);
      store_blocks<MT - NH>(acc, st, out, rows, t0, n_elem, NH, pairs, lane, j, q);
    }
  };
  for (size_t i = 0; i < R; i++) {
    const size_t t = i * W + (size_t)blockIdx.x * APPLY_WAVES + wave;
    const size_t e = t * APPLY_EPW + j;
    const bool e_ok = e < n_elem;
    half_tiles(U + (e_ok ? e : 0) * (size_t)cols, e_ok, t * APPLY_EPW);
  }
  constexpr int MTC = MT < APPLY_MTC ? MT : APPLY_MTC;
  constexpr int NC = (MT + MTC - 1) / MTC;
  if (NC > 1 && rem * NC <= W) {
    for (size_t u = kx; u < rem * NC; u += W) {
      const size_t t = R * W + u / NC;
      const int m0 = (int)(u % NC) * MTC;
      const size_t e = t * APPLY_EPW + j;
      const bool e_ok = e < n_elem;
      f32x4 acc[MTC][3];
      tile_mma_bf<L, MODE, MTC>(acc, Ab, RK, KS, RA, cols, U + (e_ok ? e : 0) * (size_t)cols, e_ok, j, q, m0, P);
      store_blocks<MTC>(acc, st, out, rows, t * APPLY_EPW, n_elem, m0, pairs, lane, j, q);
    }
  } else if (kx < rem) {
    const size_t t = R * W + kx;
    const size_t e = t * APPLY_EPW + j;
    const bool e_ok = e < n_elem;
    half_tiles(U + (e_ok ? e : 0) * (size_t)cols, e_ok, t * APPLY_EPW);
  }
}

template <class L, int MODE, int MT>
static vc_status apply_mt(const Resolved& R, const float* M, int rows, int cols, const uint64_t* U, float* out,
                          size_t n_elem, hipStream_t s)
{
  const int KS = (cols + 3) / 4;
  const int RS = apply_rs(rows);
  int dev = 0, ncu = 256;
  size_t lds_max = 64 * 1024;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      ncu = prop.multiProcessorCount;
      // the opt-in limit (160 KiB on gfx950); the default per-block limit is 64 KiB
      lds_max = prop.sharedMemPerBlockOptin > prop.sharedMemPerBlock ? prop.sharedMemPerBlockOptin
                                                                     : prop.sharedMemPerBlock;
    }
  }
  const size_t ntiles = (n_elem + APPLY_EPW - 1) / APPLY_EPW;
  size_t grid = (ntiles + APPLY_WAVES - 1) / APPLY_WAVES;
  const size_t cap = (size_t)ncu;                   // one resident workgroup per CU
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  // 8-byte stores need an even row length (3 rows) and an 8-byte aligned output
  const int pairs = (rows % 2 == 0) && (((uintptr_t)out & 7u) == 0);
  // the split-bf16 kernel where its LDS (A in three bf16 parts + block staging) fits
  if (g_apply_mode.load(std::memory_order_relaxed) == VCX_APPLY_AUTO) {
    const int KS32 = (cols + 31) / 32, RK = apply_rk(cols);
    const size_t lds_bf = (size_t)3 * (16 * MT) * RK * 2 + (size_t)APPLY_WAVES * 16 * 48 * sizeof(float);
    if (lds_bf <= lds_max) {
      const void* fb = (const void*)k_apply_bf<L, MODE, MT>;
      if (lds_bf > 64 * 1024 &&
          hipFuncSetAttribute(fb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bf) != hipSuccess)
        return VC_ERROR_HIP;
      hipLaunchKernelGGL((k_apply_bf<L, MODE, MT>), dim3((unsigned)grid), dim3(64 * APPLY_WAVES), lds_bf, s, M, rows,
                         cols, KS32, RK, U, out, n_elem, pairs, R.P);
      return launch_status();
    }
  }
  // whole-element staging where it fits beside M and `out` is 16-byte aligned
  const size_t lds_m = (size_t)4 * KS * RS * sizeof(float);
  const size_t lds_whole = lds_m + (size_t)APPLY_WAVES * apply_stage(true, rows) * sizeof(float);
  const bool whole = lds_whole <= lds_max && ((uintptr_t)out & 15u) == 0;
  const size_t lds = whole ? lds_whole : lds_m + (size_t)APPLY_WAVES * apply_stage(false, rows) * sizeof(float);
  const void* fn = whole ? (const void*)k_apply<L, MODE, MT, true> : (const void*)k_apply<L, MODE, MT, false>;
  if (lds > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return VC_ERROR_HIP;
  if (whole)
    hipLaunchKernelGGL((k_apply<L, MODE, MT, true>), dim3((unsigned)grid), dim3(64 * APPLY_WAVES), lds, s, M, rows,
                       cols, KS, RS, U, out, n_elem, pairs, R.P);
  else
    hipLaunchKernelGGL((k_apply<L, MODE, MT, false>), dim3((unsigned)grid), dim3(64 * APPLY_WAVES), lds, s, M, rows,
                       cols, KS, RS, U, out, n_elem, pairs, R.P);
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
    case 1: return apply_t<L0722, TANH>(R, M, rows, cols, U, out, n_elem, s);
    case 2: return apply_t<L0722, COS>(R, M, rows, cols, U, out, n_elem, s);
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

extern "C" vc_status vcx_set_apply_mode(int mode)
{
  if (mode != VCX_APPLY_AUTO && mode != VCX_APPLY_FP32) return VC_ERROR_INVALID_VALUE;
  g_apply_mode.store(mode, std::memory_order_relaxed);
  return VC_SUCCESS;
}

extern "C" int vcx_get_apply_mode(void) { return g_apply_mode.load(std::memory_order_relaxed); }
