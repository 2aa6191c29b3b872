// vc_fdiv.hip -- divergence of a compressed flux on hexahedral flux-reconstruction elements.
//
// Alg. (fr_fdiv_comp) of §4: every flux row F_ijp (element i, solution point j, equation p) is a
// compressed 3-vector; the divergence at point k is sum_j sum_c D[c ns + j][k] decode(F_ijp)[c].
// For the tensor-product Lagrange basis of a hexahedron (q = p + 1 Gauss-Legendre points per
// direction, j = jx + q jy + q^2 jz) the operator factors into 1D derivative matrices:
//   D[c ns + j][k] = d_c[j_c][k_c] * (the other two coordinates of j and k agree),
// so the divergence is three short line sums per point:
//   div_kp = sum_a d_0[a][kx] X_(a,ky,kz)p.x + sum_a d_1[a][ky] X_(kx,a,kz)p.y
//          + sum_a d_2[a][kz] X_(kx,ky,a)p.z.
//
// A persistent workgroup takes groups of EPW elements in turn.  For each group it
//   stages: the group's rows are contiguous, so consecutive lanes load consecutive codes; each
//      code is decoded once into LDS.  The loads of the workgroup's next group are issued right
//      after, into the same registers, and stay in flight through the three passes below;
//   x: one thread per x line of q points applies d_0 into an LDS accumulator;
//   y: adds d_1 along the y lines;
//   z: adds d_2 along the z lines and stores -- for a z line, consecutive lanes (equation, then
//      x, then y) hold consecutive outputs, so the stores are coalesced.
// The derivative coefficients are uniform across threads.  The same kernel reads plain float32
// fluxes as the uncompressed baseline.
#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

#include <type_traits>

namespace vc {

constexpr int FD_BS = 256;


template <class L, int MODE, int Q, bool CODES>
__global__ __launch_bounds__(FD_BS) void k_fdiv_tp(const float* __restrict__ d, int NP, uint32_t np_rcp,
                                                   const void* __restrict__ Fv, float* __restrict__ out,
                                                   size_t n_elem, int EPW, Params P)
{
  constexpr int Q2 = Q * Q, Q3 = Q * Q * Q;
  // EPW = FD_BS / (Q^2 NP) elements per group when that is >= 1: at most FD_BS lines and FD_BS Q
  // rows.  Only Q = 6 with NP = 8 (288 lines) falls back to one element and a loop over lines.
  constexpr bool MULTI = Q * Q * 8 > FD_BS;
  constexpr int ROWS_MAX = MULTI ? Q * Q * Q * 8 : FD_BS * Q;
  constexpr int RPT = (CODES ? 1 : 3) * ((ROWS_MAX + FD_BS - 1) / FD_BS);   // staged loads per thread
  extern __shared__ float sm[];
  const int per = Q3 * NP;
  const int gsz = EPW * per;
  float* V = sm;                              // [EPW][Q3][NP][3] decoded flux vectors
  float* Os = sm + 3 * gsz;                   // [EPW][Q3][NP] accumulator
  // Lines l = ((e Q + u) Q + v) NP + p, (u, v) the two coordinates that stay fixed along the
  // line; rows of line position a: x (a, v, u) = rx + a NP, y (v, a, u) = ry + a Q NP,
  // z (v, u, a) = rz + a Q^2 NP.
  auto bases = [&](int l, int& rx, int& ry, int& rz) {
    const int t = (int)(((uint32_t)l * np_rcp) >> 20);
    const int p = l - t * NP;
    const int v = t % Q, u = (t / Q) % Q, e = t / Q2;
    rx = (e * Q3 + Q * v + Q2 * u) * NP + p;
    ry = (e * Q3 + v + Q2 * u) * NP + p;
    rz = (e * Q3 + v + Q * u) * NP + p;
  };
  int rx0, ry0, rz0;                          // a thread's first line is the same in every group
  bases(threadIdx.x, rx0, ry0, rz0);
  auto for_lines = [&](int nlines, auto&& fn) {
    if constexpr (!MULTI) {
      if ((int)threadIdx.x < nlines) fn(rx0, ry0, rz0);
    } else {
      for (int l = threadIdx.x; l < nlines; l += FD_BS) {
        int rx, ry, rz;
        bases(l, rx, ry, rz);
        fn(rx, ry, rz);
      }
    }
  };
  // The q x q coefficients of one direction, read with scalar loads right before its pass.  The
  // empty asm hides the pointer's value from the optimiser, which would otherwise hoist all
  // 3 q^2 loads out of the group loop and spill them; the constant address space keeps the
  // reads scalar.
  auto coeffs = [&](int c, float (&dc)[Q][Q]) {
    const float* dp = d + c * Q2;
    asm volatile("" : "+s"(dp));
    typedef const __attribute__((address_space(4))) float cfloat;
    cfloat* cp = (cfloat*)dp;
#pragma unroll
    for (int a = 0; a < Q; a++)
#pragma unroll
      for (int b = 0; b < Q; b++) dc[a][b] = cp[a * Q + b];
  };
  const size_t ngroups = (n_elem + EPW - 1) / EPW;
  using R_t = typename std::conditional<CODES, uint64_t, float>::type;
  R_t r[RPT];                                 // the staged rows of the next group
  auto load = [&](size_t g) {
    const size_t e0 = g * (size_t)EPW;
    const int ne = (int)((n_elem - e0) < (size_t)EPW ? (n_elem - e0) : (size_t)EPW);
    const int cnt = CODES ? ne * per : 3 * ne * per;
    const R_t* src = (const R_t*)Fv + e0 * per * (CODES ? 1 : 3);
#pragma unroll
    for (int i = 0; i < RPT; i++) {
      const int k = (int)threadIdx.x + i * FD_BS;
      if (k < cnt) r[i] = __builtin_nontemporal_load(src + k);
    }
  };
  size_t g = blockIdx.x;
  if (g < ngroups) load(g);
  for (; g < ngroups; g += gridDim.x) {
    const size_t e0 = g * (size_t)EPW;
    const int ne = (int)((n_elem - e0) < (size_t)EPW ? (n_elem - e0) : (size_t)EPW);
    const int nlines = ne * Q2 * NP;
    float* og = out + e0 * per;
    // ---- stage: decode this group's rows into LDS, then start loading the next group, whose
    //      loads stay in flight through the three passes
    {
      const int cnt = CODES ? ne * per : 3 * ne * per;
#pragma unroll
      for (int i = 0; i < RPT; i++) {
        const int k = (int)threadIdx.x + i * FD_BS;
        if (k < cnt) {
          if constexpr (CODES) {
            float x, y, z;
            decode_vec<L, MODE>(r[i], P, x, y, z);
            V[3 * k] = x; V[3 * k + 1] = y; V[3 * k + 2] = z;
          } else {
            V[k] = r[i];
          }
        }
      }
    }
    if (g + gridDim.x < ngroups) load(g + gridDim.x);
    __syncthreads();
    // ---- x: apply d_0 along the x lines into the accumulator
    {
      float dc[Q][Q];
      coeffs(0, dc);
      for_lines(nlines, [&](int rx, int, int) {
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = V[3 * (rx + a * NP)];
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = 0.0f;
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dc[a][b], f[a], s);
          Os[rx + b * NP] = s;
        }
      });
    }
    __syncthreads();
    // ---- y: add d_1 along the y lines
    {
      float dc[Q][Q];
      coeffs(1, dc);
      for_lines(nlines, [&](int, int ry, int) {
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = V[3 * (ry + a * Q * NP) + 1];
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = 0.0f;
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dc[a][b], f[a], s);
          Os[ry + b * Q * NP] += s;
        }
      });
    }
    __syncthreads();
    // ---- z: add d_2 along the z lines and store (consecutive lanes write consecutive outputs)
    {
      float dc[Q][Q];
      coeffs(2, dc);
      for_lines(nlines, [&](int, int, int rz) {
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = V[3 * (rz + a * Q2 * NP) + 2];
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = Os[rz + b * Q2 * NP];
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dc[a][b], f[a], s);
          __builtin_nontemporal_store(s, (float*)((char*)og + (uint32_t)(rz + b * Q2 * NP) * 4u));
        }
      });
    }
    __syncthreads();   // V and Os are reused by the next group
  }
}

static inline int fdiv_epw(int q, int np)
{
  const int lines = q * q * np;
  const int e = FD_BS / lines;
  return e < 1 ? 1 : e;
}

static inline size_t fdiv_lds(int q, int np) { return (size_t)4 * fdiv_epw(q, np) * q * q * q * np * sizeof(float); }

template <class L, int MODE, int Q, bool CODES>
static vc_status fdiv_q(const Resolved& R, const float* d, int np, const void* F, float* out, size_t n_elem,
                        hipStream_t s)
{
  const int epw = fdiv_epw(Q, np);
  const size_t lds = fdiv_lds(Q, np);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_fdiv_tp<L, MODE, Q, CODES>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return VC_ERROR_HIP;
  int nb = 0, dev = 0, ncu = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fdiv_tp<L, MODE, Q, CODES>, FD_BS, lds) != hipSuccess)
    return VC_ERROR_HIP;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  const size_t groups = (n_elem + epw - 1) / epw;
  size_t grid = (size_t)ncu * (nb > 0 ? nb : 1);
  if (grid > groups) grid = groups;
  const uint32_t np_rcp = ((1u << 20) + (uint32_t)np - 1u) / (uint32_t)np;
  hipLaunchKernelGGL((k_fdiv_tp<L, MODE, Q, CODES>), dim3((unsigned)grid), dim3(FD_BS), lds, s, d, np, np_rcp, F,
                     out, n_elem, epw, R.P);
  return launch_status();
}

template <class L, int MODE, bool CODES>
static vc_status fdiv_l(const Resolved& R, const float* d, int q, int np, const void* F, float* out, size_t n_elem,
                        hipStream_t s)
{
  switch (q) {
    case 2: return fdiv_q<L, MODE, 2, CODES>(R, d, np, F, out, n_elem, s);
    case 3: return fdiv_q<L, MODE, 3, CODES>(R, d, np, F, out, n_elem, s);
    case 4: return fdiv_q<L, MODE, 4, CODES>(R, d, np, F, out, n_elem, s);
    case 5: return fdiv_q<L, MODE, 5, CODES>(R, d, np, F, out, n_elem, s);
    case 6: return fdiv_q<L, MODE, 6, CODES>(R, d, np, F, out, n_elem, s);
    default: return VC_ERROR_INVALID_VALUE;
  }
}

template <class L, int MODE, int PREC_UNUSED>
static vc_status fdiv_codes(const Resolved& R, const float* d, int q, int np, const void* F, float* out,
                            size_t n_elem, hipStream_t s)
{
  return fdiv_l<L, MODE, true>(R, d, q, np, F, out, n_elem, s);
}

static vc_status check_args(const float* d, int q, int np, const void* F, float* out, size_t n_elem, size_t align)
{
  if (q < 2 || q > 6 || np < 1 || np > 8) return VC_ERROR_INVALID_VALUE;
  if (fdiv_lds(q, np) > 80 * 1024) return VC_ERROR_INVALID_VALUE;
  if (n_elem == 0) return VC_SUCCESS;
  if (!d || !F || !out) return VC_ERROR_INVALID_VALUE;
  if (((uintptr_t)d & 3u) || ((uintptr_t)F & (align - 1)) || ((uintptr_t)out & 3u)) return VC_ERROR_MISALIGNED;
  const uintptr_t f0 = (uintptr_t)F, o0 = (uintptr_t)out;
  const size_t fb = n_elem * (size_t)q * q * q * np * (align == 8 ? 8 : 12), ob = n_elem * (size_t)q * q * q * np * 4;
  if (f0 < o0 + ob && o0 < f0 + fb) return VC_ERROR_OVERLAP;
  return VC_SUCCESS;
}

}  // namespace vc

using namespace vc;

extern "C" vc_status vc_flux_div_tp(const vc_codec* c, const float* d, int q, int np, const uint64_t* F, float* out,
                                    size_t n_elem, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  st = check_args(d, q, np, F, out, n_elem, 8);
  if (st != VC_SUCCESS || n_elem == 0) return st;
  VC_DISPATCH_NOPREC(R, fdiv_codes, R, d, q, np, F, out, n_elem, stream);
}

extern "C" vc_status vcb_flux_div_tp_f32(const float* d, int q, int np, const float* F, float* out, size_t n_elem,
                                         hipStream_t stream)
{
  vc_status st = check_args(d, q, np, F, out, n_elem, 4);
  if (st != VC_SUCCESS || n_elem == 0) return st;
  Resolved R{};
  return fdiv_l<L0722, PLAIN, false>(R, d, q, np, F, out, n_elem, stream);
}
