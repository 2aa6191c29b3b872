// vc_errhist.hip -- error statistics of the codec on the GPU, in double precision.
//
// For each input vector x (float32) the kernel runs the library's own encoder, decodes the code
// in double precision and measures the error measures of §2.2-§2.3:
//   e_vec = |x_hat - x| / |x|,  e_ang = angle(x, x_hat),  e_mag = |r_hat - |x|| / |x|
// with x_hat the FP64 decode of Eq. (a_inv)/(cart2sphere) (the inverse maps of §2.5 for the
// companded modes) and r_hat the code's exact magnitude (§2.3).  These error norms are the only
// double-precision arithmetic of the path that does not concern the encoder itself.
//
// Histograms: bin = number of edges <= e (edges ascending, FP64, staged in LDS, binary search).
// Each workgroup accumulates LDS counters and FP64 sums; a second kernel (one workgroup per
// output slot) sums the per-workgroup partials in a fixed order, so the result is deterministic.
#include <stdio.h>
#include <stdlib.h>

#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

constexpr int EH_BS = 256;
constexpr int EH_MAX_EDGES = 256;
constexpr int EH_GRID = 1024;

// inverse companding map on the signed normalised coordinate, as the encoder's forward map
template <int MODE>
__device__ __forceinline__ double hinv64(double hh, const Params& P)
{
  if constexpr (MODE == TANH) {
    const double g = (double)P.gam;
    return atanh(hh * tanh(g)) / g;
  } else {
    return asin(hh) * 0.63661977236758134;   // 2/pi
  }
}

// FP64 decode; false for the zero and reserved codes and out-of-range split fields
template <class L, int MODE>
__device__ bool decode64(uint64_t w, const Params& P, double& X, double& Y, double& Z, double& rh)
{
  const uint32_t E = (uint32_t)(w >> L::sh_e) & ((1u << L::e) - 1u);
  const uint32_t M = (uint32_t)(w >> L::sh_m) & ((1u << L::m) - 1u);
  if (E == (1u << L::e) - 1u) return false;
  if (E == 0u) {
    if (!L::keep_sub || M == 0u) return false;
    rh = ldexp((double)M, 1 - L::bias - L::m);
  } else {
    rh = ldexp(1.0 + ldexp((double)M, -L::m), (int)E - L::bias);
  }
  const uint64_t low = w & ((1ull << (L::p + L::t)) - 1ull);
  uint64_t nth, nph;
  if constexpr (MODE == FRAC) {
    if (low >= P.limit) return false;
    nph = low / P.T;
    nth = low - nph * P.T;
  } else {
    nth = low & ((1ull << L::t) - 1ull);
    nph = low >> L::t;
  }
  const double Kt = (double)P.nmax_t, Kp = (double)P.nmax_p;
  double at = (2.0 * (double)nth - Kt) / Kt;   // theta/pi
  double ap;                                    // phi/pi
  if constexpr (MODE == TANH || MODE == COS) {
    if (P.comp_t) at = hinv64<MODE>(at, P);
    ap = P.comp_p ? 0.5 * (hinv64<MODE>((2.0 * (double)nph - Kp) / Kp, P) + 1.0) : (double)nph / Kp;
  } else {
    ap = (double)nph / Kp;
  }
  double st, ct, sp, cp;
  sincospi(at, &st, &ct);
  sincospi(ap, &sp, &cp);
  X = rh * ct * sp;
  Y = rh * st * sp;
  Z = rh * cp;
  return true;
}

__device__ __forceinline__ int bin_of(double e, const double* ed, int ne)
{
  int lo = 0, hi = ne;   // first index with ed[i] > e, in [0, ne]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ed[mid] <= e) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <class L, int MODE, int PREC>
__global__ __launch_bounds__(EH_BS) void k_errhist(const float* __restrict__ xyz, size_t n,
                                                   const double* __restrict__ edges, int ne, Params P,
                                                   uint32_t* __restrict__ part_counts,
                                                   double* __restrict__ part_stats)
{
  __shared__ double ed[EH_MAX_EDGES];
  __shared__ uint32_t h[3 * (EH_MAX_EDGES + 1) + 1];
  __shared__ double red[EH_BS / 64][9];
  const int nb = ne + 1, nc = 3 * nb + 1;
  for (int i = threadIdx.x; i < ne; i += EH_BS) ed[i] = edges[i];
  for (int i = threadIdx.x; i < nc; i += EH_BS) h[i] = 0u;
  __syncthreads();

  // max of the representable magnitude and the rounding midpoint above it (clamped inputs)
  const double sat = ldexp(2.0 - ldexp(1.0, -(L::m + 1)), L::emax - L::bias);
  double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (size_t i = (size_t)blockIdx.x * EH_BS + threadIdx.x; i < n; i += (size_t)gridDim.x * EH_BS) {
    const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    const bool finite = __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
    if (!finite || (x == 0.0f && y == 0.0f && z == 0.0f)) {
      atomicAdd(&h[3 * nb], 1u);
      continue;
    }
    const double X = x, Y = y, Z = z;
    const double r = sqrt(X * X + Y * Y + Z * Z);
    const uint64_t w = encode_vec<L, MODE, PREC>(x, y, z, P);
    double xh, yh, zh, rh;
    if (r >= sat || !decode64<L, MODE>(w, P, xh, yh, zh, rh)) {
      atomicAdd(&h[3 * nb], 1u);
      continue;
    }
    const double dx = xh - X, dy = yh - Y, dz = zh - Z;
    const double cx = Y * zh - Z * yh, cy = Z * xh - X * zh, cz = X * yh - Y * xh;
    double e[3];
    e[0] = sqrt(dx * dx + dy * dy + dz * dz) / r;
    e[1] = atan2(sqrt(cx * cx + cy * cy + cz * cz), X * xh + Y * yh + Z * zh);
    e[2] = fabs(rh - r) / r;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      atomicAdd(&h[k * nb + bin_of(e[k], ed, ne)], 1u);
      s[3 * k] += e[k];
      s[3 * k + 1] += e[k] * e[k];
      s[3 * k + 2] = fmax(s[3 * k + 2], e[k]);
    }
  }
  // fixed-order workgroup reduction of the sums and maxima
#pragma unroll
  for (int k = 0; k < 9; k++) {
    double v = s[k];
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off, 64);
      v = (k % 3 == 2) ? fmax(v, o) : v + o;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int wv = 1; wv < EH_BS / 64; wv++) v = (k % 3 == 2) ? fmax(v, red[wv][k]) : v + red[wv][k];
    part_stats[(size_t)blockIdx.x * 9 + k] = v;
  }
  for (int i = threadIdx.x; i < nc; i += EH_BS) part_counts[(size_t)blockIdx.x * nc + i] = h[i];
}

// one workgroup per output slot j (counters 0 .. nc-1, then the 9 statistics): a fixed-order
// sum (or max) over the per-workgroup partials -- strided per thread, then a fixed tree
__global__ __launch_bounds__(EH_BS) void k_errhist_reduce(const uint32_t* __restrict__ part_counts,
                                                          const double* __restrict__ part_stats, int groups,
                                                          int nc, uint64_t* __restrict__ counts,
                                                          double* __restrict__ stats)
{
  __shared__ double red[EH_BS];
  const int j = blockIdx.x;
  const bool is_count = j < nc;
  const int k = j - nc;
  const bool is_max = !is_count && (k % 3 == 2);
  double v = 0.0;
  for (int g = threadIdx.x; g < groups; g += EH_BS) {
    const double p = is_count ? (double)part_counts[(size_t)g * nc + j] : part_stats[(size_t)g * 9 + k];
    v = is_max ? fmax(v, p) : v + p;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = EH_BS / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = is_max ? fmax(red[threadIdx.x], red[threadIdx.x + off])
                                                      : red[threadIdx.x] + red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (is_count) counts[j] = (uint64_t)red[0];   // exact: counts stay far below 2^53
    else stats[k] = red[0];
  }
}

template <class L, int MODE, int PREC>
static vc_status errhist_t(const Resolved& R, const float* xyz, size_t n, const double* edges, int ne,
                           uint32_t* pc, double* ps, int groups, hipStream_t s)
{
  if (groups > 0)
    hipLaunchKernelGGL((k_errhist<L, MODE, PREC>), dim3((unsigned)groups), dim3(EH_BS), 0, s, xyz, n, edges, ne,
                       R.P, pc, ps);
  return launch_status();
}

static vc_status launch_errhist(const Resolved& R, const float* xyz, size_t n, const double* edges, int ne,
                                uint32_t* pc, double* ps, int groups, hipStream_t s)
{
  VC_DISPATCH(R, errhist_t, R, xyz, n, edges, ne, pc, ps, groups, s);
}

}  // namespace vc

using namespace vc;

extern "C" vc_status vcx_error_hist(const vc_codec* c, const float* xyz, size_t n, const double* edges,
                                    int nedges, uint64_t* counts, double* stats, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (nedges < 1 || nedges > EH_MAX_EDGES || !edges || !counts || !stats) return VC_ERROR_INVALID_VALUE;
  if (n && !xyz) return VC_ERROR_INVALID_VALUE;
  if (((uintptr_t)xyz & 3u) || ((uintptr_t)edges & 7u) || ((uintptr_t)counts & 7u) || ((uintptr_t)stats & 7u))
    return VC_ERROR_MISALIGNED;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;
  const int nc = 3 * (nedges + 1) + 1;
  size_t g = (n + EH_BS - 1) / EH_BS;
  const int groups = (int)(g > (size_t)EH_GRID ? EH_GRID : g);
  uint32_t* pc = nullptr;
  double* ps = nullptr;
  const size_t bytes = (size_t)(groups ? groups : 1) * ((size_t)nc * sizeof(uint32_t) + 9 * sizeof(double));
  void* scratch = nullptr;
  const hipError_t ae = hipMallocAsync(&scratch, bytes, stream);
  if (ae != hipSuccess) {
    if (getenv("VC_LOG")) fprintf(stderr, "[vc] vcx_error_hist: hipMallocAsync(%zu) failed: %s\n", bytes, hipGetErrorString(ae));
    return ae == hipErrorOutOfMemory ? VC_ERROR_OUT_OF_MEMORY : VC_ERROR_HIP;
  }
  ps = (double*)scratch;
  pc = (uint32_t*)((char*)scratch + (size_t)(groups ? groups : 1) * 9 * sizeof(double));
  st = launch_errhist(R, xyz, n, edges, nedges, pc, ps, groups, stream);
  if (st == VC_SUCCESS) {
    hipLaunchKernelGGL(k_errhist_reduce, dim3((unsigned)(nc + 9)), dim3(EH_BS), 0, stream, (const uint32_t*)pc,
                       (const double*)ps, groups, nc, counts, stats);
    st = launch_status();
  }
  if (hipFreeAsync(scratch, stream) != hipSuccess && st == VC_SUCCESS) st = VC_ERROR_HIP;
  return st;
}
