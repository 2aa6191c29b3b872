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
// A workgroup takes EPW elements: it streams their codes (coalesced, non-temporal), decodes each
// code once into LDS (float AoS, the code order), then makes three passes -- one thread per line
// of q points -- that read q flux components and write (x pass) or add (y, z passes) q outputs
// in an LDS accumulator, which is finally stored coalesced.  The derivative coefficients are
// uniform across threads and live in scalar registers.  The same kernel reads plain float32
// fluxes as the uncompressed baseline.
#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

constexpr int FD_BS = 256;
constexpr int FD_U = 8;      // loads in flight per thread

typedef float f32x2 __attribute__((ext_vector_type(2)));

template <class L, int MODE, int Q, bool CODES>
__global__ __launch_bounds__(FD_BS) void k_fdiv_tp(const float* __restrict__ d, int NP, uint32_t np_rcp,
                                                   const void* __restrict__ Fv, float* __restrict__ out,
                                                   size_t n_elem, int EPW, Params P)
{
  constexpr int Q2 = Q * Q, Q3 = Q * Q * Q;
  extern __shared__ float sm[];
  const int per = Q3 * NP;                    // flux rows (= outputs) per element
  float* Xs = sm;                             // [EPW][Q3][NP][3]
  float* Os = sm + (size_t)3 * EPW * per;     // [EPW][Q3][NP]
  float dc[3][Q][Q];
#pragma unroll
  for (int c = 0; c < 3; c++)
#pragma unroll
    for (int a = 0; a < Q; a++)
#pragma unroll
      for (int b = 0; b < Q; b++) dc[c][a][b] = d[(c * Q + a) * Q + b];

  const size_t ngroups = (n_elem + EPW - 1) / EPW;
  for (size_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const size_t e0 = g * (size_t)EPW;
    const int ne = (int)((n_elem - e0) < (size_t)EPW ? (n_elem - e0) : (size_t)EPW);
    const int nrows = ne * per;
    // ---- load and decode: FD_U loads per thread are issued before any is used, so one memory
    // latency is paid per batch rather than per row
    if constexpr (CODES) {
      const uint64_t* F = (const uint64_t*)Fv + e0 * per;
      for (int i0 = threadIdx.x; i0 < nrows; i0 += FD_BS * FD_U) {
        uint64_t w[FD_U];
#pragma unroll
        for (int u = 0; u < FD_U; u++) {
          const int i = i0 + u * FD_BS;
          w[u] = i < nrows ? __builtin_nontemporal_load(F + i) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < FD_U; u++) {
          const int i = i0 + u * FD_BS;
          if (i < nrows) {
            float x, y, z;
            decode_vec<L, MODE>(w[u], P, x, y, z);
            Xs[3 * i] = x; Xs[3 * i + 1] = y; Xs[3 * i + 2] = z;
          }
        }
      }
    } else {
      const float* F = (const float*)Fv + e0 * per * 3;
      const int nf = 3 * nrows;
      if ((((uintptr_t)F) & 7u) == 0) {
        const f32x2* F2 = (const f32x2*)F;
        const int n2 = nf / 2;
        for (int i0 = threadIdx.x; i0 < n2; i0 += FD_BS * FD_U) {
          f32x2 v[FD_U];
#pragma unroll
          for (int u = 0; u < FD_U; u++) {
            const int i = i0 + u * FD_BS;
            v[u] = i < n2 ? __builtin_nontemporal_load(F2 + i) : f32x2{0.0f, 0.0f};
          }
#pragma unroll
          for (int u = 0; u < FD_U; u++) {
            const int i = i0 + u * FD_BS;
            if (i < n2) { Xs[2 * i] = v[u][0]; Xs[2 * i + 1] = v[u][1]; }
          }
        }
        if (threadIdx.x == 0 && (nf & 1)) Xs[nf - 1] = F[nf - 1];
      } else {
        for (int i = threadIdx.x; i < nf; i += FD_BS) Xs[i] = __builtin_nontemporal_load(F + i);
      }
    }
    __syncthreads();
    // ---- three line passes; line l = ((e Q + u) Q + v) NP + p, (u, v) the two fixed coordinates
    const int nlines = ne * Q2 * NP;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      for (int l = threadIdx.x; l < nlines; l += FD_BS) {
        // l / NP as (l * ceil(2^20 / NP)) >> 20, exact for l < 2^20 / NP (here l < 2^12)
        const int t = (int)(((uint32_t)l * np_rcp) >> 20);
        const int p = l - t * NP;
        const int v = t % Q, u = (t / Q) % Q, e = t / Q2;
        // point index of line position a: x pass (a, v, u), y pass (v, a, u), z pass (v, u, a)
        const int base = e * Q3 + (c == 0 ? Q * v + Q2 * u : c == 1 ? v + Q2 * u : v + Q * u);
        const int stride = c == 0 ? 1 : c == 1 ? Q : Q2;
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = Xs[((base + a * stride) * NP + p) * 3 + c];
#pragma unroll
        for (int b = 0; b < Q; b++) {
          float s = 0.0f;
#pragma unroll
          for (int a = 0; a < Q; a++) s = __builtin_fmaf(dc[c][a][b], f[a], s);
          float* o = Os + (base + b * stride) * NP + p;
          *o = c == 0 ? s : *o + s;
        }
      }
      __syncthreads();
    }
    // ---- store
    float* og = out + e0 * per;
    for (int i = threadIdx.x; i < nrows; i += FD_BS) __builtin_nontemporal_store(Os[i], og + i);
    __syncthreads();   // Xs / Os are reused by the next group
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
