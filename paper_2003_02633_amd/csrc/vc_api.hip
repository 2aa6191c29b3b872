// vc_api.hip -- C ABI of libvc: argument validation, codec resolution, dispatch.
#include <math.h>
#include <mutex>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vc_internal.hpp"
#include "vc_params.hpp"
#include "../../include/vc_ext.h"

namespace vc {

static inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// the result of an empty reduction, written by a kernel (not a memset node, so that a caller may
// capture the call in a graph)
__global__ void k_zero_result(float* out) { out[0] = 0.0f; }

static bool overlaps(const void* p, size_t pb, const void* q, size_t qb)
{
  uintptr_t a0 = (uintptr_t)p, a1 = a0 + pb, b0 = (uintptr_t)q, b1 = b0 + qb;
  return a0 < b1 && b0 < a1;
}

// VC_LOG set to a non-empty value other than "0": each core entry point writes one line to stderr
// when it returns (its codec, size, the axpy launch configuration, the status).  Read once.
static bool log_on()
{
  static const bool on = [] {
    const char* e = getenv("VC_LOG");
    return e && *e && strcmp(e, "0") != 0;
  }();
  return on;
}

static vc_status logged(const char* fn, const vc_codec* c, size_t n, vc_status st)
{
  if (log_on()) {
    char cfg[64] = "";
    if (strcmp(fn, "vc_axpy") == 0 && c && c->struct_size == sizeof(vc_codec)) {
      const StreamCfg g = stream_cfg(c->precision == VC_PREC_F32 ? PREC_F32 : PREC_F64);
      const bool tuned = c->layout == VC_LAYOUT_0_7_22_17_18 && c->mode == VC_MODE_PLAIN && c->mag_round == VC_MAG_RNE;
      snprintf(cfg, sizeof cfg, " block=%d pairs/lane=%d nt=%d", tuned ? g.block : 512, tuned ? g.vpt : 2,
               tuned ? g.nt : 1);
    }
    if (c && c->struct_size == sizeof(vc_codec))
      fprintf(stderr, "[vc] %s n=%zu layout=%u mode=%u mag_round=%u precision=%u%s -> %s\n", fn, n, c->layout,
              c->mode, c->mag_round, c->precision, cfg, vc_status_string(st));
    else
      fprintf(stderr, "[vc] %s n=%zu (no valid codec) -> %s\n", fn, n, vc_status_string(st));
  }
  return st;
}

}  // namespace vc

using namespace vc;

extern "C" {

vc_status vc_codec_init(vc_codec* c, const char* layout)
{
  if (!c) return VC_ERROR_INVALID_VALUE;
  int lay = VC_LAYOUT_0_7_22_17_18;
  if (layout) {
    lay = -1;
    for (const auto& L : kLayouts)
      if (strcmp(L.name, layout) == 0) lay = L.layout;
    if (lay < 0) return VC_ERROR_UNSUPPORTED_CODEC;
  }
  memset(c, 0, sizeof(*c));
  c->struct_size = sizeof(vc_codec);
  c->layout = (uint32_t)lay;
  c->mode = VC_MODE_PLAIN;
  c->mag_round = VC_MAG_RNE;
  c->compand_mask = VC_COMPAND_PHI | VC_COMPAND_THETA;
  c->gamma = 0.5f;
  c->frac_P = 1ull << 17;
  c->precision = VC_PREC_F64;
  return VC_SUCCESS;
}

static vc_status encode_impl(const vc_codec* c, const float* xyz, uint64_t* codes, size_t n, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (n == 0) return VC_SUCCESS;
  if (!xyz || !codes) return VC_ERROR_INVALID_VALUE;
  if (!aligned(xyz, 4) || !aligned(codes, 8)) return VC_ERROR_MISALIGNED;
  if (overlaps(xyz, 12 * n, codes, 8 * n)) return VC_ERROR_OVERLAP;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;
  return launch_encode(R, xyz, codes, n, stream);
}

vc_status vc_encode(const vc_codec* c, const float* xyz, uint64_t* codes, size_t n, hipStream_t stream)
{
  return logged("vc_encode", c, n, encode_impl(c, xyz, codes, n, stream));
}

static vc_status decode_impl(const vc_codec* c, const uint64_t* codes, float* xyz, size_t n, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (n == 0) return VC_SUCCESS;
  if (!xyz || !codes) return VC_ERROR_INVALID_VALUE;
  if (!aligned(xyz, 4) || !aligned(codes, 8)) return VC_ERROR_MISALIGNED;
  if (overlaps(xyz, 12 * n, codes, 8 * n)) return VC_ERROR_OVERLAP;
  return launch_decode(R, codes, xyz, n, stream);
}

vc_status vc_decode(const vc_codec* c, const uint64_t* codes, float* xyz, size_t n, hipStream_t stream)
{
  return logged("vc_decode", c, n, decode_impl(c, codes, xyz, n, stream));
}

static vc_status axpy_common(const vc_codec* c, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* out,
                             size_t n, float* dump, hipStream_t stream)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (n == 0) return VC_SUCCESS;
  if (!a || !b || !out) return VC_ERROR_INVALID_VALUE;
  if (!aligned(a, 8) || !aligned(b, 8) || !aligned(out, 8)) return VC_ERROR_MISALIGNED;
  if ((out != a && overlaps(out, 8 * n, a, 8 * n)) || (out != b && overlaps(out, 8 * n, b, 8 * n)))
    return VC_ERROR_OVERLAP;
  if (dump && !aligned(dump, 4)) return VC_ERROR_MISALIGNED;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;
  return launch_axpy(R, alpha, a, b, out, n, dump, stream);
}

// public precision (vc_precision) -> device Prec index; -1 = both
static int prec_index(int precision)
{
  if (precision < 0) return -1;
  return precision == VC_PREC_F64 ? PREC_F64 : precision == VC_PREC_F32 ? PREC_F32 : -2;
}

vc_status vcx_set_stream_config(int precision, int block, int vpt, int nt)
{
  const int p = prec_index(precision);
  if (p < -1 || (vpt != 2 && vpt != 4 && vpt != 8)) return VC_ERROR_UNSUPPORTED_CODEC;
  return set_axpy_cfg(p, block, vpt / 2, nt);
}

vc_status vcx_get_stream_config(int precision, int* block, int* vpt, int* nt)
{
  if (!block || !vpt || !nt) return VC_ERROR_INVALID_VALUE;
  const int p = prec_index(precision);
  if (p < 0) return VC_ERROR_UNSUPPORTED_CODEC;
  const StreamCfg g = stream_cfg(p);
  *block = g.block;
  *vpt = 2 * g.vpt;
  *nt = g.nt;
  return VC_SUCCESS;
}

vc_status vcx_load_tuning(const char* path)
{
  if (!path) return VC_ERROR_INVALID_VALUE;
  FILE* f = fopen(path, "r");
  if (!f) return VC_ERROR_INVALID_VALUE;
  char line[256];
  vc_status st = VC_SUCCESS;
  while (fgets(line, sizeof line, f) && st == VC_SUCCESS) {
    int b = 0, v = 0, t = 0;
    char prec[8] = {0};
    if (sscanf(line, "axpy %7s block=%d vpt=%d nt=%d", prec, &b, &v, &t) == 4) {
      const int p = strcmp(prec, "f64") == 0 ? VC_PREC_F64 : strcmp(prec, "f32") == 0 ? VC_PREC_F32 : -2;
      st = p == -2 ? VC_ERROR_INVALID_VALUE : vcx_set_stream_config(p, b, v, t);
    } else if (sscanf(line, "axpy block=%d vpt=%d nt=%d", &b, &v, &t) == 3) {
      st = vcx_set_stream_config(-1, b, v, t);
    } else if (sscanf(line, "batch ua=%d ud=%d un=%d", &b, &v, &t) == 3) {
      st = vcx_set_batch_config(b, v, t);
    }
  }
  fclose(f);
  return st;
}

static void apply_env_tuning()
{
  static std::once_flag once;                     // the first vc_axpy call of any thread
  std::call_once(once, [] {
    const char* p = getenv("VC_TUNE_CACHE");
    if (p && *p) (void)vcx_load_tuning(p);
  });
}

vc_status vc_axpy(const vc_codec* c, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n,
                  hipStream_t stream)
{
  apply_env_tuning();
  return logged("vc_axpy", c, n, axpy_common(c, alpha, a, b, out, n, nullptr, stream));
}

vc_status vcx_axpy_dump(const vc_codec* c, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* out,
                        float* c32, size_t n, hipStream_t stream)
{
  if (n && !c32) return VC_ERROR_INVALID_VALUE;
  return logged("vcx_axpy_dump", c, n, axpy_common(c, alpha, a, b, out, n, c32, stream));
}

// Partial sums of vc_dot_noalloc, one float per reduction block.  reduce_parts(n) never exceeds
// kScratchSlots, so every n fits.  Each device holds its own copy of the array (8 KiB) until the
// process ends; in host code `scratch` only names the symbol, so kernels get the device address
// that hipGetSymbolAddress returns, looked up once per device with that device current.
constexpr int kScratchSlots = 2048;
static __device__ __align__(256) float scratch[kScratchSlots];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch[kMaxDevices];

static vc_status scratch_on_current_device(float** out)
{
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VC_ERROR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    float* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return VC_ERROR_HIP;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return VC_SUCCESS;
}

static vc_status reduce_common(const vc_codec* c, const uint64_t* a, const uint64_t* b, size_t n, float* d_out,
                               hipStream_t stream, bool is_dot, bool noalloc = false)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if (!d_out) return VC_ERROR_INVALID_VALUE;
  if (!aligned(d_out, 4)) return VC_ERROR_MISALIGNED;
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(1), 0, stream, d_out);
    return launch_status();
  }
  if (!a || (is_dot && !b)) return VC_ERROR_INVALID_VALUE;
  if (!aligned(a, 8) || (is_dot && !aligned(b, 8))) return VC_ERROR_MISALIGNED;
  const int np = reduce_parts(n);
  float* parts = nullptr;
  if (noalloc) {
    if (np > kScratchSlots) return VC_ERROR_INVALID_VALUE;
    st = scratch_on_current_device(&parts);
    if (st != VC_SUCCESS) return st;
    return is_dot ? launch_dot(R, a, b, n, parts, np, d_out, stream) : launch_norm2(R, a, n, parts, np, d_out, stream);
  }
  const hipError_t ae = hipMallocAsync((void**)&parts, sizeof(float) * np, stream);
  if (ae != hipSuccess) return ae == hipErrorOutOfMemory ? VC_ERROR_OUT_OF_MEMORY : VC_ERROR_HIP;
  st = is_dot ? launch_dot(R, a, b, n, parts, np, d_out, stream) : launch_norm2(R, a, n, parts, np, d_out, stream);
  if (hipFreeAsync(parts, stream) != hipSuccess && st == VC_SUCCESS) st = VC_ERROR_HIP;
  return st;
}

vc_status vcx_inline_params(const vc_codec* c, void* params, size_t size)
{
  if (!params || size != sizeof(Params)) return VC_ERROR_INVALID_VALUE;
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;
  memcpy(params, &R.P, sizeof(Params));
  return VC_SUCCESS;
}

size_t vcx_inline_params_size(void) { return sizeof(Params); }

vc_status vc_dot(const vc_codec* c, const uint64_t* a, const uint64_t* b, size_t n, float* d_out,
                 hipStream_t stream)
{
  return logged("vc_dot", c, n, reduce_common(c, a, b, n, d_out, stream, true));
}

vc_status vc_dot_noalloc(const vc_codec* c, const uint64_t* a, const uint64_t* b, size_t n, float* d_out,
                         hipStream_t stream)
{
  return logged("vc_dot_noalloc", c, n, reduce_common(c, a, b, n, d_out, stream, true, true));
}

vc_status vc_norm2(const vc_codec* c, const uint64_t* a, size_t n, float* d_out, hipStream_t stream)
{
  return logged("vc_norm2", c, n, reduce_common(c, a, nullptr, n, d_out, stream, false));
}

const char* vc_status_string(vc_status s)
{
  switch (s) {
    case VC_SUCCESS: return "VC_SUCCESS";
    case VC_ERROR_INVALID_VALUE: return "VC_ERROR_INVALID_VALUE";
    case VC_ERROR_MISALIGNED: return "VC_ERROR_MISALIGNED";
    case VC_ERROR_UNSUPPORTED_CODEC: return "VC_ERROR_UNSUPPORTED_CODEC";
    case VC_ERROR_LAUNCH: return "VC_ERROR_LAUNCH";
    case VC_ERROR_HIP: return "VC_ERROR_HIP";
    case VC_ERROR_OUT_OF_MEMORY: return "VC_ERROR_OUT_OF_MEMORY";
    case VC_ERROR_OVERLAP: return "VC_ERROR_OVERLAP";
    default: return "VC_ERROR_UNKNOWN";
  }
}

const char* vc_version(void) { return "libvc 0.1 (gfx950)"; }

}  // extern "C"
