// vc_batch.hip -- batched persistent launch over a segment table, replayed from a HIP graph.
//
// Many short streaming operations (axpy, dot, norm2, encode on independent arrays) are the
// typical shape of a solver step; launched one by one, each pays a launch and a ramp-up/drain
// of the whole chip.  Here every segment is cut into tiles (a tile size per operation, see
// BatchCfg), numbered consecutively segment after segment, and ONE persistent kernel walks the
// tile range with a static grid stride.  A workgroup's tile index only grows, so its segment
// cursor only moves forward (at most nseg steps over the whole launch).
//
// dot / norm2 tiles write one FP32 partial per wave (a fixed-order in-wave sum) into per-tile
// slots; a second kernel sums each reduction segment's slots in index order and writes the
// result.  Every slot that the second kernel reads is written by the first, so nothing needs
// clearing (no memset node in the graph), and results are deterministic.
#include <algorithm>
#include <atomic>
#include <type_traits>
#include <new>
#include <vector>

#include "vc_internal.hpp"
#include "../../include/vc_ext.h"

namespace vc {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BB = 256;                    // threads per workgroup (four waves)

// Tile shape per operation, in code pairs per lane: axpy UA, dot UD, norm2 UN (a tile is
// 512 U vectors); encode tiles are 1024 vectors (each wave stages 256 float vectors through LDS).
// Chosen by the autotuner for the default codec; process-wide, read when a plan is created.
struct BatchCfg {
  int ua, ud, un;
};
static std::atomic<uint32_t> g_batch_cfg{2u | 4u << 8 | 8u << 16};

static BatchCfg batch_cfg()
{
  const uint32_t v = g_batch_cfg.load(std::memory_order_relaxed);
  return {(int)(v & 0xffu), (int)((v >> 8) & 0xffu), (int)((v >> 16) & 0xffu)};
}

struct BatchSeg {
  uint32_t op;          // vc_op
  uint32_t vec_ok;      // all pointers allow the 16-byte code path / 16-byte float path
  float alpha;
  uint32_t tile_shift;  // log2 of the vectors per tile of this segment's operation
  uint64_t n;
  uint64_t tile0;       // global index of the segment's first tile
  const void* a;
  const void* b;
  void* out;
  uint64_t pad2;
};
static_assert(sizeof(BatchSeg) == 64, "segment record is one 64-byte line");

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One persistent kernel over the tiles of all segments.  Vectorised tiles move every wave's
// accesses as 1 KiB contiguous 16-byte loads/stores (codes: wave w of a tile takes U 128-code
// steps, lane l the pair at 2l of each; floats: three 16-byte accesses per lane into LDS); the
// last, partial tile of a segment and unaligned segments go one vector per thread.  dot / norm2
// tiles leave one partial per wave, with no barrier.
template <class L, int MODE, int PREC, int UA, int UD, int UN>
__global__ __launch_bounds__(BB) void k_batch(const BatchSeg* __restrict__ segs, int nseg, size_t total_tiles,
                                              float* __restrict__ parts, Params P0)
{
  __shared__ float stage[BB / 64][256 * 3];
  with_compand_mask<MODE>(P0, [&](const Params& P) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int s = 0;
  for (size_t t = blockIdx.x; t < total_tiles; t += gridDim.x) {
    while (s + 1 < nseg && segs[s + 1].tile0 <= t) s++;
    const BatchSeg S = segs[s];
    const size_t tv = (size_t)1 << S.tile_shift;
    const size_t v0 = (t - S.tile0) << S.tile_shift;
    const bool vec = S.vec_ok && v0 + tv <= S.n;
    if (S.op == VC_OP_AXPY) {
      const uint64_t* a = (const uint64_t*)S.a;
      const uint64_t* b = (const uint64_t*)S.b;
      uint64_t* c = (uint64_t*)S.out;
      if (vec) {
        const size_t i0 = v0 + (size_t)wv * (UA * 128) + 2 * lane;
        u64x2 va[UA], vb[UA];
#pragma unroll
        for (int u = 0; u < UA; u++) {
          va[u] = __builtin_nontemporal_load((const u64x2*)(a + i0 + 128 * u));
          vb[u] = __builtin_nontemporal_load((const u64x2*)(b + i0 + 128 * u));
        }
#pragma unroll
        for (int u = 0; u < UA; u++) {
          u64x2 o;
#pragma unroll
          for (int h = 0; h < 2; h++) {
            float ax, ay, az, bx, by, bz;
            decode_vec<L, MODE>(va[u][h], P, ax, ay, az);
            decode_vec<L, MODE>(vb[u][h], P, bx, by, bz);
            o[h] = encode_vec<L, MODE, PREC>(__builtin_fmaf(S.alpha, ax, bx), __builtin_fmaf(S.alpha, ay, by),
                                             __builtin_fmaf(S.alpha, az, bz), P);
          }
          __builtin_nontemporal_store(o, (u64x2*)(c + i0 + 128 * u));
        }
      } else {
        for (size_t i = v0 + threadIdx.x; i < v0 + tv && i < S.n; i += BB) {
          float ax, ay, az, bx, by, bz;
          decode_vec<L, MODE>(a[i], P, ax, ay, az);
          decode_vec<L, MODE>(b[i], P, bx, by, bz);
          c[i] = encode_vec<L, MODE, PREC>(__builtin_fmaf(S.alpha, ax, bx), __builtin_fmaf(S.alpha, ay, by),
                                           __builtin_fmaf(S.alpha, az, bz), P);
        }
      }
    } else if (S.op == VC_OP_ENCODE) {
      const float* x = (const float*)S.a;
      uint64_t* c = (uint64_t*)S.out;
      if (vec) {
        // wave wv: vectors w0 .. w0 + 255; lane l encodes 2l, 2l + 1, 128 + 2l, 129 + 2l
        const size_t w0 = v0 + 256 * (size_t)wv;
        float* sw = stage[wv];
        const f32x4* src = (const f32x4*)(x + 3 * w0);
        f32x4 q[3];
#pragma unroll
        for (int k = 0; k < 3; k++) q[k] = __builtin_nontemporal_load(src + 64 * k + lane);
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
        o0[0] = encode_vec<L, MODE, PREC>(v[0], v[1], v[2], P);
        o0[1] = encode_vec<L, MODE, PREC>(v[3], v[4], v[5], P);
        o1[0] = encode_vec<L, MODE, PREC>(v[6], v[7], v[8], P);
        o1[1] = encode_vec<L, MODE, PREC>(v[9], v[10], v[11], P);
        u64x2* dst = (u64x2*)(c + w0);
        __builtin_nontemporal_store(o0, dst + lane);
        __builtin_nontemporal_store(o1, dst + 64 + lane);
      } else {
        for (size_t i = v0 + threadIdx.x; i < v0 + tv && i < S.n; i += BB)
          c[i] = encode_vec<L, MODE, PREC>(x[3 * i], x[3 * i + 1], x[3 * i + 2], P);
      }
    } else {   // VC_OP_DOT, VC_OP_NORM2: one partial per wave
      const uint64_t* a = (const uint64_t*)S.a;
      const uint64_t* b = (const uint64_t*)S.b;
      float acc = 0.0f;
      if (S.op == VC_OP_DOT) {
        if (vec) {
          const size_t i0 = v0 + (size_t)wv * (UD * 128) + 2 * lane;
          u64x2 va[UD], vb[UD];
#pragma unroll
          for (int u = 0; u < UD; u++) {
            va[u] = __builtin_nontemporal_load((const u64x2*)(a + i0 + 128 * u));
            vb[u] = __builtin_nontemporal_load((const u64x2*)(b + i0 + 128 * u));
          }
#pragma unroll
          for (int u = 0; u < UD; u++)
#pragma unroll
            for (int h = 0; h < 2; h++) acc += dot_pair<L, MODE>(va[u][h], vb[u][h], P);
        } else {
          for (size_t i = v0 + threadIdx.x; i < v0 + tv && i < S.n; i += BB) acc += dot_pair<L, MODE>(a[i], b[i], P);
        }
      } else {
        if (vec) {
          const size_t i0 = v0 + (size_t)wv * (UN * 128) + 2 * lane;
          u64x2 va[UN];
#pragma unroll
          for (int u = 0; u < UN; u++) va[u] = __builtin_nontemporal_load((const u64x2*)(a + i0 + 128 * u));
#pragma unroll
          for (int u = 0; u < UN; u++)
#pragma unroll
            for (int h = 0; h < 2; h++) {
              const float r = decode_mag_checked<L, MODE>(va[u][h], P);
              acc = __builtin_fmaf(r, r, acc);
            }
        } else {
          for (size_t i = v0 + threadIdx.x; i < v0 + tv && i < S.n; i += BB) {
            const float r = decode_mag_checked<L, MODE>(a[i], P);
            acc = __builtin_fmaf(r, r, acc);
          }
        }
      }
      const float sum = wave_sum(acc);
      if (lane == 0) parts[4 * t + wv] = sum;
    }
  }
  });
}

// one workgroup per segment: the fixed-order sum of a reduction segment's wave partials
__global__ __launch_bounds__(BB) void k_batch_reduce(const BatchSeg* __restrict__ segs,
                                                     const float* __restrict__ parts)
{
  __shared__ float red[BB / 64];
  const BatchSeg S = segs[blockIdx.x];
  if (S.op != VC_OP_DOT && S.op != VC_OP_NORM2) return;
  const size_t np = 4 * (((S.n + ((size_t)1 << S.tile_shift) - 1)) >> S.tile_shift);
  float acc = 0.0f;
  for (size_t i = threadIdx.x; i < np; i += BB) acc += parts[4 * S.tile0 + i];
  const float w = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < BB / 64; i++) sum += red[i];
    *(float*)S.out = sum;
  }
}

template <class L, int MODE, int PREC, int UA, int UD, int UN>
static vc_status batch_launch_t(const Resolved& R, const BatchSeg* segs, int nseg, size_t total_tiles, float* parts,
                                unsigned grid, hipStream_t s)
{
  if (total_tiles)
    hipLaunchKernelGGL((k_batch<L, MODE, PREC, UA, UD, UN>), dim3(grid), dim3(BB), 0, s, segs, nseg, total_tiles,
                       parts, R.P);
  vc_status st = launch_status();
  if (st != VC_SUCCESS) return st;
  hipLaunchKernelGGL(k_batch_reduce, dim3((unsigned)nseg), dim3(BB), 0, s, segs, (const float*)parts);
  return launch_status();
}

template <class L, int MODE, int PREC, int UA, int UD, int UN>
static vc_status batch_occ_t(unsigned* blocks_per_cu)
{
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<L, MODE, PREC, UA, UD, UN>, BB, 0) != hipSuccess)
    return VC_ERROR_HIP;
  *blocks_per_cu = nb > 0 ? (unsigned)nb : 1u;
  return VC_SUCCESS;
}

// tile shapes built: the tuned set for the default codec (ua 1-2, ud 2-8, un 4-16), (2, 4, 8) for
// the others
#define VC_BATCH_UN(FN, L, MODE, PREC, UA, UD, G, ...)                                    \
  switch (G.un) {                                                                         \
    case 4: return FN<L, MODE, PREC, UA, UD, 4>(__VA_ARGS__);                             \
    case 8: return FN<L, MODE, PREC, UA, UD, 8>(__VA_ARGS__);                             \
    default: return FN<L, MODE, PREC, UA, UD, 16>(__VA_ARGS__);                           \
  }
#define VC_BATCH_UD(FN, L, MODE, PREC, UA, G, ...)                                        \
  switch (G.ud) {                                                                         \
    case 2: VC_BATCH_UN(FN, L, MODE, PREC, UA, 2, G, __VA_ARGS__)                         \
    case 4: VC_BATCH_UN(FN, L, MODE, PREC, UA, 4, G, __VA_ARGS__)                         \
    default: VC_BATCH_UN(FN, L, MODE, PREC, UA, 8, G, __VA_ARGS__)                        \
  }
#define VC_BATCH_SHAPES(FN, L, MODE, PREC, G, ...)                                        \
  if constexpr (std::is_same<L, L0722>::value && MODE == PLAIN) {                         \
    if (G.ua == 1) { VC_BATCH_UD(FN, L, MODE, PREC, 1, G, __VA_ARGS__) }                  \
    else { VC_BATCH_UD(FN, L, MODE, PREC, 2, G, __VA_ARGS__) }                            \
  } else {                                                                                \
    return FN<L, MODE, PREC, 2, 4, 8>(__VA_ARGS__);                                       \
  }

template <class L, int MODE, int PREC>
static vc_status batch_launch(const Resolved& R, BatchCfg G, const BatchSeg* segs, int nseg, size_t total_tiles,
                              float* parts, unsigned grid, hipStream_t s)
{
  VC_BATCH_SHAPES(batch_launch_t, L, MODE, PREC, G, R, segs, nseg, total_tiles, parts, grid, s)
}

template <class L, int MODE, int PREC>
static vc_status batch_grid(BatchCfg G, unsigned* blocks_per_cu)
{
  VC_BATCH_SHAPES(batch_occ_t, L, MODE, PREC, G, blocks_per_cu)
}

static vc_status launch_batch(const Resolved& R, BatchCfg G, const BatchSeg* segs, int nseg, size_t total_tiles,
                              float* parts, unsigned grid, hipStream_t s)
{
  VC_DISPATCH(R, batch_launch, R, G, segs, nseg, total_tiles, parts, grid, s);
}

static vc_status occupancy(const Resolved& R, BatchCfg G, unsigned* blocks_per_cu)
{
  VC_DISPATCH(R, batch_grid, G, blocks_per_cu);
}

// the shape a plan uses: the process-wide configuration for the default codec, else (2, 4, 8)
static BatchCfg plan_cfg(const Resolved& R)
{
  if (R.layout == VC_LAYOUT_0_7_22_17_18 && R.mode == VC_MODE_PLAIN && R.mag_round == VC_MAG_RNE) return batch_cfg();
  return {2, 4, 8};
}

static uint32_t tile_shift(uint32_t op, BatchCfg G)
{
  const int u = op == VC_OP_AXPY ? G.ua : op == VC_OP_DOT ? G.ud : op == VC_OP_NORM2 ? G.un : 2;
  return (uint32_t)(__builtin_ctz((unsigned)u) + 9);   // 512 u vectors (encode: 1024)
}

}  // namespace vc

using namespace vc;

struct vc_batch_plan {
  Resolved R;
  int device = 0;
  int nseg = 0;
  std::vector<vc_segment> segs;
  std::vector<size_t> sep_off;     // per segment: first partial slot of the separate-launch path
  BatchSeg* d_segs = nullptr;
  BatchCfg cfg = {2, 4, 8};        // tile shape (read from the process-wide configuration)
  float* d_parts = nullptr;        // four slots (one per wave) per tile (persistent path)
  float* d_sep_parts = nullptr;    // reduce_parts(n) slots per reduction segment (separate path)
  size_t total_tiles = 0;
  unsigned grid = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t sep_graph = nullptr;
  hipGraphExec_t sep_exec = nullptr;
};

namespace {

struct Span {
  uintptr_t lo, hi;
  int seg;
};

bool overlap(uintptr_t a0, size_t ab, uintptr_t b0, size_t bb) { return a0 < b0 + bb && b0 < a0 + ab; }

// per-segment checks, and: no segment writes memory that another segment reads or writes
// (the persistent kernel runs all segments' tiles concurrently, in no fixed order)
vc_status validate(const vc_segment* segs, int nseg)
{
  std::vector<Span> writes, reads;
  for (int i = 0; i < nseg; i++) {
    const vc_segment& S = segs[i];
    const uintptr_t a = (uintptr_t)S.a, b = (uintptr_t)S.b, o = (uintptr_t)S.out;
    const uint64_t n = S.n;
    if (n > (1ull << 40)) return VC_ERROR_INVALID_VALUE;
    switch (S.op) {
      case VC_OP_AXPY:
        if (n == 0) continue;
        if (!a || !b || !o) return VC_ERROR_INVALID_VALUE;
        if ((a | b | o) & 7u) return VC_ERROR_MISALIGNED;
        if ((o != a && overlap(o, 8 * n, a, 8 * n)) || (o != b && overlap(o, 8 * n, b, 8 * n)))
          return VC_ERROR_OVERLAP;
        writes.push_back({o, o + 8 * n, i});
        reads.push_back({a, a + 8 * n, i});
        reads.push_back({b, b + 8 * n, i});
        break;
      case VC_OP_ENCODE:
        if (n == 0) continue;
        if (!a || !o) return VC_ERROR_INVALID_VALUE;
        if ((a & 3u) || (o & 7u)) return VC_ERROR_MISALIGNED;
        if (overlap(a, 12 * n, o, 8 * n)) return VC_ERROR_OVERLAP;
        writes.push_back({o, o + 8 * n, i});
        reads.push_back({a, a + 12 * n, i});
        break;
      case VC_OP_DOT:
      case VC_OP_NORM2:
        if (!o) return VC_ERROR_INVALID_VALUE;
        if (o & 3u) return VC_ERROR_MISALIGNED;
        writes.push_back({o, o + 4, i});
        if (n == 0) continue;
        if (!a || (S.op == VC_OP_DOT && !b)) return VC_ERROR_INVALID_VALUE;
        if ((a & 7u) || (S.op == VC_OP_DOT && (b & 7u))) return VC_ERROR_MISALIGNED;
        reads.push_back({a, a + 8 * n, i});
        if (S.op == VC_OP_DOT) reads.push_back({b, b + 8 * n, i});
        break;
      default:
        return VC_ERROR_INVALID_VALUE;
    }
  }
  std::sort(writes.begin(), writes.end(), [](const Span& x, const Span& y) { return x.lo < y.lo; });
  for (size_t k = 1; k < writes.size(); k++)
    if (writes[k].lo < writes[k - 1].hi) return VC_ERROR_OVERLAP;
  // writes are disjoint and sorted, so their ends are sorted too
  for (const Span& r : reads) {
    auto it = std::upper_bound(writes.begin(), writes.end(), r.lo,
                               [](uintptr_t v, const Span& w) { return v < w.hi; });
    for (; it != writes.end() && it->lo < r.hi; ++it)
      if (it->seg != r.seg) return VC_ERROR_OVERLAP;
  }
  return VC_SUCCESS;
}

vc_status run_separate_launches(vc_batch_plan* p, hipStream_t s)
{
  for (int i = 0; i < p->nseg; i++) {
    const vc_segment& S = p->segs[i];
    vc_status st = VC_SUCCESS;
    switch (S.op) {
      case VC_OP_AXPY:
        if (S.n) st = launch_axpy(p->R, S.alpha, (const uint64_t*)S.a, (const uint64_t*)S.b, (uint64_t*)S.out, S.n,
                                  nullptr, s);
        break;
      case VC_OP_ENCODE:
        if (S.n) st = launch_encode(p->R, (const float*)S.a, (uint64_t*)S.out, S.n, s);
        break;
      case VC_OP_DOT:
        st = launch_dot(p->R, (const uint64_t*)S.a, (const uint64_t*)S.b, S.n, p->d_sep_parts + p->sep_off[i],
                        reduce_parts(S.n), (float*)S.out, s);
        break;
      case VC_OP_NORM2:
        st = launch_norm2(p->R, (const uint64_t*)S.a, S.n, p->d_sep_parts + p->sep_off[i], reduce_parts(S.n),
                          (float*)S.out, s);
        break;
    }
    if (st != VC_SUCCESS) return st;
  }
  return VC_SUCCESS;
}

void release(vc_batch_plan* p)
{
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->sep_exec) (void)hipGraphExecDestroy(p->sep_exec);
  if (p->sep_graph) (void)hipGraphDestroy(p->sep_graph);
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->d_parts) (void)hipFree(p->d_parts);
  if (p->d_sep_parts) (void)hipFree(p->d_sep_parts);
  delete p;
}

// capture `fn(plan, capture_stream)` into a graph and instantiate it
template <class F>
vc_status capture(vc_batch_plan* p, F fn, hipGraph_t* g, hipGraphExec_t* e)
{
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return VC_ERROR_HIP;
  vc_status st = VC_SUCCESS;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = VC_ERROR_HIP;
  } else {
    st = fn(p, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (st == VC_SUCCESS && ee != hipSuccess) st = VC_ERROR_HIP;
    if (st == VC_SUCCESS && hipGraphInstantiate(e, graph, nullptr, nullptr, 0) != hipSuccess) st = VC_ERROR_HIP;
    if (st == VC_SUCCESS) *g = graph;
    else if (graph) (void)hipGraphDestroy(graph);
  }
  (void)hipStreamDestroy(cs);
  return st;
}

}  // namespace

extern "C" {

vc_status vc_batch_plan_create(vc_batch_plan** plan, const vc_codec* c, const vc_segment* segs, int nseg,
                               hipStream_t stream)
{
  if (!plan) return VC_ERROR_INVALID_VALUE;
  *plan = nullptr;
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (nseg < 0 || nseg > (1 << 20) || (nseg > 0 && !segs)) return VC_ERROR_INVALID_VALUE;
  st = validate(segs, nseg);
  if (st != VC_SUCCESS) return st;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;     // axpy and encode segments encode

  vc_batch_plan* p = new (std::nothrow) vc_batch_plan;
  if (!p) return VC_ERROR_OUT_OF_MEMORY;
  p->R = R;
  p->cfg = plan_cfg(R);
  p->nseg = nseg;
  p->segs.assign(segs, segs + nseg);
  (void)hipGetDevice(&p->device);

  std::vector<BatchSeg> h(nseg);
  size_t tiles = 0, sep = 0;
  p->sep_off.assign(nseg, 0);
  for (int i = 0; i < nseg; i++) {
    const vc_segment& S = segs[i];
    BatchSeg& B = h[i];
    B = BatchSeg{};
    B.op = S.op;
    B.alpha = S.alpha;
    B.n = S.n;
    B.tile0 = tiles;
    B.a = S.a;
    B.b = S.b;
    B.out = S.out;
    const uintptr_t a = (uintptr_t)S.a, b = (uintptr_t)S.b, o = (uintptr_t)S.out;
    if (S.op == VC_OP_ENCODE) B.vec_ok = ((a | o) & 15u) == 0;
    else if (S.op == VC_OP_AXPY) B.vec_ok = ((a | b | o) & 15u) == 0;
    else if (S.op == VC_OP_DOT) B.vec_ok = ((a | b) & 15u) == 0;
    else B.vec_ok = (a & 15u) == 0;
    B.tile_shift = tile_shift(S.op, p->cfg);
    tiles += (S.n + ((uint64_t)1 << B.tile_shift) - 1) >> B.tile_shift;
    if (S.op == VC_OP_DOT || S.op == VC_OP_NORM2) {
      p->sep_off[i] = sep;
      sep += (size_t)reduce_parts(S.n);
    }
  }
  p->total_tiles = tiles;

  unsigned per_cu = 1;
  int ncu = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) ncu = prop.multiProcessorCount;
  st = occupancy(R, p->cfg, &per_cu);
  if (st == VC_SUCCESS) {
    size_t g = (size_t)ncu * per_cu;
    if (g > tiles) g = tiles;
    p->grid = g < 1 ? 1u : (unsigned)g;
  }

  if (st == VC_SUCCESS && nseg > 0) {
    if (hipMalloc((void**)&p->d_segs, sizeof(BatchSeg) * nseg) != hipSuccess ||
        hipMalloc((void**)&p->d_parts, 4 * sizeof(float) * (tiles ? tiles : 1)) != hipSuccess ||
        hipMalloc((void**)&p->d_sep_parts, sizeof(float) * (sep ? sep : 1)) != hipSuccess)
      st = VC_ERROR_OUT_OF_MEMORY;
    else if (hipMemcpyAsync(p->d_segs, h.data(), sizeof(BatchSeg) * nseg, hipMemcpyHostToDevice, stream) !=
                 hipSuccess ||
             hipStreamSynchronize(stream) != hipSuccess)
      st = VC_ERROR_HIP;
  }
  if (st == VC_SUCCESS && nseg > 0)
    st = capture(p,
                 [](vc_batch_plan* q, hipStream_t cs) {
                   return launch_batch(q->R, q->cfg, q->d_segs, q->nseg, q->total_tiles, q->d_parts, q->grid, cs);
                 },
                 &p->graph, &p->exec);
  if (st != VC_SUCCESS) {
    release(p);
    return st;
  }
  *plan = p;
  return VC_SUCCESS;
}

vc_status vc_batch_plan_run(vc_batch_plan* p, hipStream_t stream)
{
  if (!p) return VC_ERROR_INVALID_VALUE;
  if (p->nseg == 0) return VC_SUCCESS;
  return hipGraphLaunch(p->exec, stream) == hipSuccess ? VC_SUCCESS : VC_ERROR_LAUNCH;
}

vc_status vc_batch_plan_run_separate(vc_batch_plan* p, hipStream_t stream)
{
  if (!p) return VC_ERROR_INVALID_VALUE;
  return run_separate_launches(p, stream);
}

vc_status vcx_batch_plan_run_separate_graph(vc_batch_plan* p, hipStream_t stream)
{
  if (!p) return VC_ERROR_INVALID_VALUE;
  if (p->nseg == 0) return VC_SUCCESS;
  if (!p->sep_exec) {
    vc_status st = capture(p, run_separate_launches, &p->sep_graph, &p->sep_exec);
    if (st != VC_SUCCESS) return st;
  }
  return hipGraphLaunch(p->sep_exec, stream) == hipSuccess ? VC_SUCCESS : VC_ERROR_LAUNCH;
}

vc_status vcx_batch_plan_info(const vc_batch_plan* p, uint64_t* total_tiles, uint32_t* grid)
{
  if (!p || !total_tiles || !grid) return VC_ERROR_INVALID_VALUE;
  *total_tiles = p->total_tiles;
  *grid = p->grid;
  return VC_SUCCESS;
}

vc_status vcx_set_batch_config(int ua, int ud, int un)
{
  const bool ok = (ua == 1 || ua == 2) && (ud == 2 || ud == 4 || ud == 8) && (un == 4 || un == 8 || un == 16);
  if (!ok) return VC_ERROR_UNSUPPORTED_CODEC;
  g_batch_cfg.store((uint32_t)ua | (uint32_t)ud << 8 | (uint32_t)un << 16, std::memory_order_relaxed);
  return VC_SUCCESS;
}

vc_status vcx_get_batch_config(int* ua, int* ud, int* un)
{
  if (!ua || !ud || !un) return VC_ERROR_INVALID_VALUE;
  const BatchCfg G = batch_cfg();
  *ua = G.ua;
  *ud = G.ud;
  *un = G.un;
  return VC_SUCCESS;
}

vc_status vc_batch_plan_destroy(vc_batch_plan* p)
{
  if (!p) return VC_SUCCESS;
  release(p);
  return VC_SUCCESS;
}

}  // extern "C"
