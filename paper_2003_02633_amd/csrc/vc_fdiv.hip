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
// A workgroup takes EPW elements and makes three passes, one thread per line of q points:
//   x: load the line's q codes (all in flight at once), decode each once, apply d_0 into an LDS
//      accumulator and keep the y and z components in LDS;
//   y: add d_1 along the y lines;
//   z: add d_2 along the z lines and store -- for a z line, consecutive lanes (equation, then x,
//      then y) hold consecutive outputs, so the stores are coalesced.
// The derivative coefficients are uniform across threads.  The same kernel reads plain float32
// fluxes as the uncompressed baseline.
#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

constexpr int FD_BS = 256;


template <class L, int MODE, int Q, bool CODES>
__global__ __launch_bounds__(FD_BS) void k_fdiv_tp(const float* __restrict__ d, int NP, uint32_t np_rcp,
                                                   const void* __restrict__ Fv, float* __restrict__ out,
                                                   size_t n_elem, int EPW, Params P)
{
  constexpr int Q2 = Q * Q, Q3 = Q * Q * Q;
  extern __shared__ float sm[];
  const int per = Q3 * NP;                    // flux rows (= outputs) per element
  float* Ys = sm;                             // [EPW][Q3][NP] y components
  float* Zs = sm + (size_t)EPW * per;         // [EPW][Q3][NP] z components
  float* Os = sm + (size_t)2 * EPW * per;     // [EPW][Q3][NP] accumulator
  // the 3 q x q derivative coefficients, staged once; each pass reads its own q x q block with
  // uniform (broadcast) LDS reads right before use, so only q^2 of them are live at a time
  __shared__ float dsh[3 * Q2];
  for (int i = threadIdx.x; i < 3 * Q2; i += FD_BS) dsh[i] = d[i];
  __syncthreads();
  // Lines l = ((e Q + u) Q + v) NP + p, (u, v) the two coordinates that stay fixed along the
  // line; rows of line position a: x (a, v, u) = rx + a NP, y (v, a, u) = ry + a Q NP,
  // z (v, u, a) = rz + a Q^2 NP.
  auto bases = [&](int l, int& rx, int& ry, int& rz) {
    const int t = (int)(((uint32_t)l * np_rcp) >> 20);   // l / NP, exact for l < 2^20 / NP
    const int p = l - t * NP;
    const int v = t % Q, u = (t / Q) % Q, e = t / Q2;
    rx = (e * Q3 + Q * v + Q2 * u) * NP + p;
    ry = (e * Q3 + v + Q2 * u) * NP + p;
    rz = (e * Q3 + v + Q * u) * NP + p;
  };
  // a thread's first line (l = threadIdx.x) is the same in every group: its bases are computed once
  int rx0, ry0, rz0;
  bases(threadIdx.x, rx0, ry0, rz0);

  const size_t ngroups = (n_elem + EPW - 1) / EPW;
  for (size_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const size_t e0 = g * (size_t)EPW;
    const int ne = (int)((n_elem - e0) < (size_t)EPW ? (n_elem - e0) : (size_t)EPW);
    const int nlines = ne * Q2 * NP;
    const uint64_t* Fc = (const uint64_t*)Fv + e0 * per;    // this group's rows (uniform base)
    const float* Ff = (const float*)Fv + e0 * per * 3;
    float* og = out + e0 * per;

    // ---- x: load and decode a line of q rows, apply d_0, keep y and z for the other passes
    {
      float dx[Q][Q];   // this pass's coefficients (uniform LDS reads)
#pragma unroll
      for (int a = 0; a < Q; a++)
#pragma unroll
        for (int b = 0; b < Q; b++) dx[a][b] = dsh[a * Q + b];
      auto xline = [&](int r0) {
        float fx[Q];
        if constexpr (CODES) {
          uint64_t w[Q];
#pragma unroll
          for (int a = 0; a < Q; a++)
            w[a] = __builtin_nontemporal_load((const uint64_t*)((const char*)Fc + (uint32_t)(r0 + a * NP) * 8u));
#pragma unroll
          for (int a = 0; a < Q; a++) {
            float y, z;
            decode_vec<L, MODE>(w[a], P, fx[a], y, z);
            Ys[r0 + a * NP] = y;
            Zs[r0 + a * NP] = z;
          }
        } else {
          float y[Q], z[Q];
#pragma unroll
          for (int a = 0; a < Q; a++) {
            const float* f = (const float*)((const char*)Ff + (uint32_t)(r0 + a * NP) * 12u);
            fx[a] = __builtin_nontemporal_load(f);
            y[a] = __builtin_nontemporal_load(f + 1);
            z[a] = __builtin_nontemporal_load(f + 2);
          }
#pragma unroll
          for (int a = 0; a < Q; a++) { Ys[r0 + a * NP] = y[a]; Zs[r0 + a * NP] = z[a]; }
        }
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = 0.0f;
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dx[a][b], fx[a], s);
          Os[r0 + b * NP] = s;
        }
      };
      for (int l = threadIdx.x; l < nlines; l += FD_BS) {
        int rx = rx0, ry = ry0, rz = rz0;
        if (l != (int)threadIdx.x) bases(l, rx, ry, rz);
        xline(rx);
      }
    }
    __syncthreads();
    // ---- y: add d_1 along the y lines
    {
      float dy[Q][Q];
#pragma unroll
      for (int a = 0; a < Q; a++)
#pragma unroll
        for (int b = 0; b < Q; b++) dy[a][b] = dsh[Q2 + a * Q + b];
      auto yline = [&](int r0) {
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = Ys[r0 + a * Q * NP];
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = 0.0f;
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dy[a][b], f[a], s);
          Os[r0 + b * Q * NP] += s;
        }
      };
      for (int l = threadIdx.x; l < nlines; l += FD_BS) {
        int rx = rx0, ry = ry0, rz = rz0;
        if (l != (int)threadIdx.x) bases(l, rx, ry, rz);
        yline(ry);
      }
    }
    __syncthreads();
    // ---- z: add d_2 along the z lines and store (consecutive lanes write consecutive outputs)
    {
      float dz[Q][Q];
#pragma unroll
      for (int a = 0; a < Q; a++)
#pragma unroll
        for (int b = 0; b < Q; b++) dz[a][b] = dsh[2 * Q2 + a * Q + b];
      auto zline = [&](int r0) {
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = Zs[r0 + a * Q2 * NP];
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = Os[r0 + b * Q2 * NP];
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dz[a][b], f[a], s);
          __builtin_nontemporal_store(s, (float*)((char*)og + (uint32_t)(r0 + b * Q2 * NP) * 4u));
        }
      };
      for (int l = threadIdx.x; l < nlines; l += FD_BS) {
        int rx = rx0, ry = ry0, rz = rz0;
        if (l != (int)threadIdx.x) bases(l, rx, ry, rz);
        zline(rz);
      }
    }
    __syncthreads();   // Ys / Zs / Os are reused by the next group
  }
}

static inline int fdiv_epw(int q, int np)
{
  const int lines = q * q * np;
  const int e = FD_BS / lines;
  return e < 1 ? 1 : e;
}

static inline size_t fdiv_lds(int q, int np) { return (size_t)3 * fdiv_epw(q, np) * q * q * q * np * sizeof(float); }

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
